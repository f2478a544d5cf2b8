// Hidden pre-activations theta = W s + b on MFMA, with tanh in the epilogue,
// and ln psi(s).
//
// The contraction Theta[r][j] = sum_i s~[r][i] W~^T[i][j] (s~ augmented with a
// 1 at i = N so that row N of W~^T adds b) runs on CDNA4 matrix cores:
//   FP64 path: v_mfma_f64_16x16x4f64,
//   FP32 path: v_mfma_f32_16x16x4f32,
//   BF16 form: v_mfma_f32_16x16x32_bf16 twice (W = W_hi + W_lo, both BF16,
//              spins exact), FP32 accumulation.
// Operand lane layouts (16x16 tiles, 64 lanes): A[row = lane % 16][k = lane / 16]
// (BF16: k = 8 * (lane / 16) + e), B[k][col = lane % 16]; accumulator slot i
// of lane l holds D[acc_row(l / 16, i)][l % 16] (see common.h).
// One workgroup = 4 waves = 64 rows x 64 hidden columns; each wave owns 16 rows.
#include "kernels.h"

namespace nqs {

template <typename R>
__device__ __forceinline__ R act(R th, int col, int M) {
    return col < M ? (R)tanh(th) : (col == M ? (R)1 : (R)0);
}

template <typename R>
__device__ __forceinline__ R spin_aug(const int8_t* __restrict__ s, int N, int r, int rows, int k) {
    if (r >= rows || k > N) return (R)0;
    return k == N ? (R)1 : (R)s[(size_t)r * N + k];
}

// Block = 4 waves = 64 rows x 64 hidden columns.  The sites run in tiles of
// TK_THETA: each tile's spins (augmented, [64][TK]) and the block's 64 columns
// of W~^T ([TK][64]) are staged in LDS with batched loads, then every wave runs
// its 16 rows over the tile (any lattice size fits the fixed LDS footprint).
constexpr int TK_THETA = 128;

template <typename R>
__global__ __launch_bounds__(256) void k_theta(Dims d, const int8_t* __restrict__ s, int rows,
                                               const R* __restrict__ Wa, R* __restrict__ dst1,
                                               R* __restrict__ dst2, long dst2_stride) {
    constexpr int TK = TK_THETA;
    __shared__ __align__(16) R Bs[TK * 64];     // [TK][64]
    __shared__ __align__(16) int8_t Ss[64 * TK];  // [64][TK]
    const int Na = d.Na;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int rowb = blockIdx.x * 64, row0 = rowb + wave * 16;
    const int col0 = blockIdx.y * 64;
    typedef typename std::conditional<sizeof(R) == 8, v4d, v4f>::type acc_t;
    acc_t acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = acc_t{0, 0, 0, 0};
    for (int kt = 0; kt < Na; kt += TK) {
        const int kn = min(TK, Na - kt);  // a multiple of 16 (Na is)
        __syncthreads();                  // the previous tile is no longer read
        for (int base = 0; base < kn * 64; base += 256 * 8) {
            R v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = base + u * 256 + tid;
                const int k = e >> 6, cl = e & 63;
                v[u] = (e < kn * 64 && col0 + cl < d.Mw) ? Wa[(size_t)(kt + k) * d.Mw + col0 + cl]
                                                         : (R)0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = base + u * 256 + tid;
                if (e < kn * 64) Bs[e] = v[u];
            }
        }
        for (int base = 0; base < 64 * kn; base += 256 * 8) {
            int8_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = base + u * 256 + tid;
                const int rl = e / kn, k = e - rl * kn;
                v[u] = (e < 64 * kn) ? (int8_t)spin_aug<R>(s, d.N, rowb + rl, rows, kt + k)
                                     : (int8_t)0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = base + u * 256 + tid;
                if (e < 64 * kn) Ss[e] = v[u];
            }
        }
        __syncthreads();
        const int8_t* Sw = Ss + (wave * 16 + lr) * kn;
        for (int k0 = 0; k0 < kn; k0 += 4) {
            const R a = (R)Sw[k0 + lk];
            const R* Bk = Bs + (k0 + lk) * 64 + lr;
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const R b = Bk[ct * 16];
                if constexpr (sizeof(R) == 8)
                    acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[ct], 0, 0, 0);
                else
                    acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[ct], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int col = col0 + ct * 16 + lr;
        if (col >= d.Mw) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = row0 + acc_row<R>(lk, i);
            if (row >= rows) continue;
            const R t = act<R>(acc[ct][i], col, d.M);
            dst1[(size_t)row * d.Mw + col] = t;
            if (dst2) dst2[(size_t)row * dst2_stride + col] = t;
        }
    }
}

typedef short v8s __attribute__((ext_vector_type(8)));

// BF16 form: spins are exact in BF16 (+1 = 0x3F80, -1 = 0xBF80).
__device__ __forceinline__ v8bf spins_bf16(const int8_t* __restrict__ s, int N, int r, int rows,
                                           int k0) {
    v8s v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = k0 + e;
        short bits = 0;
        if (r < rows && k <= N) {
            const int sv = k == N ? 1 : (int)s[(size_t)r * N + k];
            bits = sv > 0 ? (short)0x3F80 : (short)0xBF80;
        }
        v[e] = bits;
    }
    return __builtin_bit_cast(v8bf, v);
}

constexpr int TB_KC = 64;            // k per LDS chunk (two k-steps of 32)
constexpr int TB_LD = TB_KC + 8;     // LDS row of one column (+8: spreads the banks)

__global__ __launch_bounds__(256) void k_theta_bf16(Dims d, const int8_t* __restrict__ s, int rows,
                                                    const uint16_t* __restrict__ Whi,
                                                    const uint16_t* __restrict__ Wlo,
                                                    float* __restrict__ dst1, float* __restrict__ dst2,
                                                    long dst2_stride) {
    // block = 64 rows x 64 columns, wave = 16 rows x the 64 columns (four MFMA
    // tiles sharing the spin fragment).  The block's W panel moves through LDS
    // in chunks of 64 k (two coalesced 16-byte loads per thread and plane, read
    // by all four waves); the next chunk's W and spins are in flight while the
    // current chunk is multiplied.  Per element the accumulation order is that
    // of one k-step at a time: + a W_hi, then + a W_lo.
    __shared__ __attribute__((aligned(16))) uint16_t Sh[2][64 * TB_LD];
    __shared__ __attribute__((aligned(16))) uint16_t Sl[2][64 * TB_LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int row0 = blockIdx.x * 64 + wave * 16;
    const int col0 = blockIdx.y * 64;
    const int nch = (d.Kb + TB_KC - 1) / TB_KC;
    // staging items of this thread: columns sc and sc + 32 of the panel, k
    // offset sk of the chunk (8 entries each)
    const int sc = tid >> 3, sk = (tid & 7) * 8;
    const bool scin0 = col0 + sc < d.Mw, scin1 = col0 + sc + 32 < d.Mw;
    const uint16_t* gh = Whi + (size_t)(col0 + sc) * d.Kb + sk;
    const uint16_t* gl = Wlo + (size_t)(col0 + sc) * d.Kb + sk;
    const size_t g32 = (size_t)32 * d.Kb;  // 32 columns further
    const v8s z8 = {0, 0, 0, 0, 0, 0, 0, 0};
    v4f acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = v4f{0, 0, 0, 0};
    v8s nh, nl, nh1, nl1;
    v8bf na[2];
    auto fetch = [&](int ch) {  // W pieces of chunk ch, and this lane's spins for it
        const int k = ch * TB_KC + sk;
        const bool kin = k < d.Kb;
        nh = (scin0 && kin) ? *(const v8s*)(gh + ch * TB_KC) : z8;
        nl = (scin0 && kin) ? *(const v8s*)(gl + ch * TB_KC) : z8;
        nh1 = (scin1 && kin) ? *(const v8s*)(gh + g32 + ch * TB_KC) : z8;
        nl1 = (scin1 && kin) ? *(const v8s*)(gl + g32 + ch * TB_KC) : z8;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int kk = ch * TB_KC + 32 * u + 8 * lk;
            na[u] = kk < d.Kb ? spins_bf16(s, d.N, row0 + lr, rows, kk)
                              : __builtin_bit_cast(v8bf, z8);
        }
    };
    fetch(0);
    *(v8s*)&Sh[0][sc * TB_LD + sk] = nh;
    *(v8s*)&Sl[0][sc * TB_LD + sk] = nl;
    *(v8s*)&Sh[0][(sc + 32) * TB_LD + sk] = nh1;
    *(v8s*)&Sl[0][(sc + 32) * TB_LD + sk] = nl1;
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const v8bf a0 = na[0], a1 = na[1];
        if (ch + 1 < nch) fetch(ch + 1);
        const uint16_t* ph = Sh[ch & 1];
        const uint16_t* pl = Sl[ch & 1];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const v8bf a = u == 0 ? a0 : a1;
            if (ch * TB_KC + 32 * u < d.Kb) {
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    const int o = (ct * 16 + lr) * TB_LD + 32 * u + 8 * lk;
                    const v8s bh = *(const v8s*)&ph[o], bl = *(const v8s*)&pl[o];
                    acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(v8bf, bh),
                                                                      acc[ct], 0, 0, 0);
                    acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(v8bf, bl),
                                                                      acc[ct], 0, 0, 0);
                }
            }
        }
        if (ch + 1 < nch) {
            *(v8s*)&Sh[(ch + 1) & 1][sc * TB_LD + sk] = nh;
            *(v8s*)&Sl[(ch + 1) & 1][sc * TB_LD + sk] = nl;
            *(v8s*)&Sh[(ch + 1) & 1][(sc + 32) * TB_LD + sk] = nh1;
            *(v8s*)&Sl[(ch + 1) & 1][(sc + 32) * TB_LD + sk] = nl1;
        }
        __syncthreads();
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int col = col0 + ct * 16 + lr;
        if (col >= d.Mw) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = row0 + acc_row<float>(lk, i);
            if (row >= rows) continue;
            const float t = act<float>(acc[ct][i], col, d.M);
            dst1[(size_t)row * d.Mw + col] = t;
            if (dst2) dst2[(size_t)row * dst2_stride + col] = t;
        }
    }
}

// ln psi(s) = sum_i a_i s_i + sum_j ln cosh theta_j; one wave per configuration.
template <typename R>
__global__ __launch_bounds__(256) void k_log_psi(Dims d, const double* __restrict__ Pm,
                                                 const R* __restrict__ Wa,
                                                 const int8_t* __restrict__ s, long n,
                                                 R* __restrict__ out) {
    const long r = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    const int8_t* sr = s + r * d.N;
    R acc = 0;
    for (int j = lane; j < d.M; j += 64) {
        R th = Wa[(size_t)d.N * d.Mw + j];
        for (int i = 0; i < d.N; ++i) th += (R)sr[i] * Wa[(size_t)i * d.Mw + j];
        const R ath = th < 0 ? -th : th;
        // ln cosh x = |x| + ln(1 + e^{-2|x|}) - ln 2, finite for any x
        acc += ath + (R)log1p(exp(-2 * ath)) - (R)0.69314718055994530942;
    }
    if (d.vb)
        for (int i = lane; i < d.N; i += 64) acc += (R)(Pm[(size_t)d.M * d.Na + i] * sr[i]);
    acc = wave_sum(acc);
    if (lane == 0) out[r] = acc;
}

void launch_theta(hipStream_t st, const Dims& d, int prec, const Tables& t, const int8_t* s,
                  int rows, void* dst1, void* dst2, long dst2_stride) {
    if (rows <= 0) return;
    dim3 grid((rows + 63) / 64, (d.Mw + 63) / 64);
    if (prec == 0)
        k_theta<double><<<grid, 256, 0, st>>>(d, s, rows, (const double*)t.Wa, (double*)dst1,
                                              (double*)dst2, dst2_stride);
    else if (prec == 1)
        k_theta<float><<<grid, 256, 0, st>>>(d, s, rows, (const float*)t.Wa, (float*)dst1,
                                             (float*)dst2, dst2_stride);
    else
        k_theta_bf16<<<grid, 256, 0, st>>>(d, s, rows, t.Whi, t.Wlo, (float*)dst1, (float*)dst2,
                                           dst2_stride);
}

void launch_log_psi(hipStream_t st, const Dims& d, int prec, const double* Pm, const Tables& t,
                    const int8_t* s, long n, void* out) {
    if (n <= 0) return;
    const int nb = (int)((n + 3) / 4);
    if (prec == 0)
        k_log_psi<double><<<nb, 256, 0, st>>>(d, Pm, (const double*)t.Wa, s, n, (double*)out);
    else
        k_log_psi<float><<<nb, 256, 0, st>>>(d, Pm, (const float*)t.Wa, s, n, (float*)out);
}

}  // namespace nqs
