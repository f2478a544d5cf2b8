// Force and on-the-fly QGT products of one SR step, and the CG iteration
// that uses them (paper: force-vector equation; QGT estimator equation;
// appendix "QGTOnTheFly"; section "Solving linear systems").
//
// With the augmented layout (common.h) the log-derivatives of sample k are the
// outer product t~_k (x) s~_k, so
//   contraction 1:  w_k = t~_k . (P s~_k)                (w = J p)
//   contraction 2:  out = sum_k z_k t~_k (x) s~_k        (out = J^T z)
// with z = (w - mean w) / N_s for the QGT product (G p = J^T dw) and
// z = 2 (E - mean E) / N_s for the force.
//
// Once per SR step the batch is laid out for the matrix cores with the
// contracted (sample or site) index contiguous:
//   Sp  augmented spins, sample-major (contraction 1)
//   St  augmented spins, site-major   (contraction 2)
//       (int8 on the FP64 path; in the BF16 forms one FP4 (E2M1) code per
//       spin, +1 = 0x2, -1 = 0xA, padding 0, so that one conversion
//       instruction turns two spins into two exact BF16 values)
//   Th  [Ma][Nsp]       t~ hidden-major (FP64 path: double; BF16 forms: float)
// FP64 path: v_mfma_f64_16x16x4f64.  FP32/BF16 forms: v_mfma_f32_16x16x32_bf16
// with FP32 accumulation and spins exact in BF16 (+1 / -1); the real-valued
// operand is an FP32 quantity split into two BF16 terms (x = hi + lo), each
// term contracted with the spins: contraction 1 the CG residual (the update
// writes it split), contraction 2 the FP32 product t~ z formed while the tile
// is staged.
//
// No kernel here uses atomics or fences: every reduction is a fixed-order
// sum of per-block partials done by the consumer kernel (each block of the
// consumer recomputes the same sum), and block 0 publishes the CG scalars for
// the host.
#include "kernels.h"

#include <type_traits>
#include <algorithm>
#include <utility>

namespace nqs {

typedef short v8s __attribute__((ext_vector_type(8)));

__device__ __forceinline__ double bsum256(double v, double* sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}


// ---------------------------------------------------------------------------
// per-step layout kernels
// ---------------------------------------------------------------------------
// FP64 path: int8 spins, Sp [Nsp][Kq] and St [Kb][Nsp] (the constant column
// i = N holds 1; padding rows and columns 0, whose products are zero or
// discarded).
__global__ __launch_bounds__(256) void k_prep_spins(const int8_t* __restrict__ s, int N, long n,
                                                    int Kb, int Kq, long Nsp,
                                                    int8_t* __restrict__ Sp,
                                                    int8_t* __restrict__ St) {
    __shared__ int8_t tile[64][68];
    const long k0 = (long)blockIdx.x * 64;
    const int i0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int kl = e >> 6, il = e & 63;
        const long k = k0 + kl;
        const int i = i0 + il;
        int8_t v = 0;
        if (k < n) v = i < N ? s[k * N + i] : (i == N ? (int8_t)1 : (int8_t)0);
        tile[kl][il] = v;
        if (i < Kq) Sp[k * Kq + i] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int il = e >> 6, kl = e & 63;
        const int i = i0 + il;
        if (i < Kb) St[(long)i * Nsp + k0 + kl] = tile[kl][il];
    }
}

// ---------------------------------------------------------------------------
// BF16 forms: spins as FP4 (E2M1) codes, two per byte (element 2m in the low
// nibble of byte m).  Sites are stored in an order that makes each lane's
// operand run contiguous: within a group of 128 sites, site 32 u + 8 q + e
// (u, q < 4, e < 8) sits at position 32 q + 8 u + e (bit fields 3-4 and 5-6
// swapped), so that lane quad q reads the 32 codes of its four k-steps u in
// one 16-byte load.  In the site-major copy the samples of each 512-sample
// chunk are ordered the same way: local sample 32 u + 8 q + e (u < 16) sits
// at position 128 q + 8 u + e.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fp4_code(int s) { return s > 0 ? 0x2u : (s < 0 ? 0xAu : 0u); }

typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
// 8 FP4 spin codes (one 32-bit word) as 8 BF16 values (+1, -1 or 0), exact
__device__ __forceinline__ v8bf fp4x8_to_bf16(uint32_t x) {
    uint4 r;
    r.x = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(x, 1.0f, 0));
    r.y = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(x, 1.0f, 1));
    r.z = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(x, 1.0f, 2));
    r.w = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(x, 1.0f, 3));
    return __builtin_bit_cast(v8bf, r);
}
__device__ __forceinline__ uint32_t word_of(const uint4& v, int u) {
    return u == 0 ? v.x : (u == 1 ? v.y : (u == 2 ? v.z : v.w));
}

// Two FP32 values as the BF16 pairs hi (round to nearest even) and
// lo = bf16(x - hi), each packed two to a 32-bit word (element 0 low).
__device__ __forceinline__ void split_pk(float x0, float x1, uint32_t& hi, uint32_t& lo) {
    v2bf h;
    h[0] = (__bf16)x0;
    h[1] = (__bf16)x1;
    hi = __builtin_bit_cast(uint32_t, h);
    v2bf l;
    l[0] = (__bf16)(x0 - __uint_as_float(hi << 16));
    l[1] = (__bf16)(x1 - __uint_as_float(hi & 0xFFFF0000u));
    lo = __builtin_bit_cast(uint32_t, l);
}

// Contraction-1 operands of the BF16 forms in matrix-core fragment order, so
// that every load instruction of a wave reads 1 KB of contiguous memory:
//   residual (two BF16 planes): entry (j, i) of plane h at
//     ((((j / 16) * (Kq / 128) + i / 128) * 4 + u) * 64 + 16 q + j % 16) * 8 + e,
//     with i % 128 = 32 u + 8 q + e (the operand of lane 16 q + j % 16 in k-step u);
//   activations: t~ of sample k = 64 b + 16 rt + r and hidden unit
//     j = 16 c + 4 q + v at (((b * (Ma / 16) + c) * 4 + rt) * 64 + 16 q + r) * 4 + v
//     (the four hidden rows lane 16 q + r of hidden tile c needs for sample tile rt).
__host__ __device__ __forceinline__ size_t pfrag_off(int j, int i, int ng) {
    const int l = i & 127;
    return ((((size_t)(j >> 4) * ng + (i >> 7)) * 4 + (l >> 5)) * 64 + 16 * ((l >> 3) & 3) +
            (j & 15)) * 8 + (l & 7);
}

// BF16 forms: Sp [Nsp][Kq / 2] bytes (sample-major, sites in the order above) and
// St [Kb][Nsp / 2] bytes (site-major, samples of each chunk in the order
// above).  One block: 64 samples x one 128-site group, staged in LDS.
__global__ __launch_bounds__(256) void k_prep_spins4(const int8_t* __restrict__ s, int N, long n,
                                                     int Kb, int Kq, long Nsp,
                                                     uint8_t* __restrict__ Sp,
                                                     uint8_t* __restrict__ St) {
    __shared__ int8_t tile[64][132];
    const long k0 = (long)blockIdx.x * 64;
    const int i0 = blockIdx.y * 128;
    for (int e = threadIdx.x; e < 64 * 128; e += 256) {
        const int kl = e >> 7, il = e & 127;
        const long k = k0 + kl;
        const int i = i0 + il;
        int8_t v = 0;
        if (k < n) v = i < N ? s[k * N + i] : (i == N ? (int8_t)1 : (int8_t)0);
        tile[kl][il] = v;
    }
    __syncthreads();
    {   // sample-major: thread -> sample kl, positions 32 q .. 32 q + 31 (16 bytes)
        const int kl = threadIdx.x >> 2, q = threadIdx.x & 3;
        uint32_t wv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            uint32_t x = 0;
#pragma unroll
            for (int e = 0; e < 8; ++e) x |= fp4_code(tile[kl][32 * u + 8 * q + e]) << (4 * e);
            wv[u] = x;  // positions 32 q + 8 u + e
        }
        *(uint4*)(Sp + (k0 + kl) * (Kq / 2) + i0 / 2 + 16 * q) = make_uint4(wv[0], wv[1], wv[2], wv[3]);
    }
    {   // site-major: thread -> site il, lane quads q = 2 h, 2 h + 1: positions
        // 128 q + 16 a + (0..15) of the chunk hold local samples 32 (2 a + (p >> 3)) + 8 q + (p & 7)
        const int il = threadIdx.x >> 1, h = threadIdx.x & 1;
        const int i = i0 + il;
        if (i < Kb) {
            const long c0 = k0 & ~511L;         // chunk start
            const int a = (int)((k0 & 511) >> 6);  // which 64-sample slice of the chunk
#pragma unroll
            for (int qq = 0; qq < 2; ++qq) {
                const int q = 2 * h + qq;
                uint32_t x0 = 0, x1 = 0;
#pragma unroll
                for (int p = 0; p < 16; ++p) {
                    const int kl = 32 * (p >> 3) + 8 * q + (p & 7);  // sample k0 + kl
                    const uint32_t c = fp4_code(tile[kl][il]);
                    if (p < 8) x0 |= c << (4 * p);
                    else x1 |= c << (4 * (p - 8));
                }
                *(uint2*)(St + (size_t)i * (Nsp / 2) + c0 / 2 + 64 * q + 8 * a) = make_uint2(x0, x1);
            }
        }
    }
}

// t~ hidden-major: Th[j][k] = t~_kj (k < Nsp, padding samples 0), in the
// compute precision (FP64 path: double; BF16 forms: float).
template <typename R>
__global__ __launch_bounds__(256) void k_prep_t(const R* __restrict__ tact, long n, int Mw, int Ma,
                                                long Nsp, void* __restrict__ out) {
    __shared__ R tile[64][65];
    const long k0 = (long)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int kl = e >> 6, jl = e & 63;
        const long k = k0 + kl;
        const int j = j0 + jl;
        tile[kl][jl] = (k < n && j < Ma) ? tact[k * Mw + j] : (R)0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int jl = e >> 6, kl = e & 63;
        const int j = j0 + jl;
        if (j >= Ma) continue;
        const size_t o = (size_t)j * Nsp + k0 + kl;
        ((R*)out)[o] = tile[kl][jl];
    }
}

// BF16 forms: the activations in contraction-1 fragment order (zero past n).
// Block (b, c): 64 samples x hidden tile c; thread = (sample tile, lane).
__global__ __launch_bounds__(256) void k_prep_tf(const float* __restrict__ tact, long n, int Mw,
                                                 float* __restrict__ Tf) {
    const int b = blockIdx.x, c = blockIdx.y, nct = gridDim.y;
    const int rt = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const long k = 64L * b + 16 * rt + r;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (k < n) v = *(const float4*)(tact + k * Mw + 16 * c + 4 * q);
    *(float4*)(Tf + ((((size_t)b * nct + c) * 4 + rt) * 64 + lane) * 4) = v;
}

// ---------------------------------------------------------------------------
// CG iteration it runs in three kernels: contraction 1 (with the CG "head"),
// contraction 2, and the update.  Standard CG steps, arranged so that no
// kernel forms the direction for the matrix cores:
//   w_it = J p_it = J r_it + beta_it w_{it-1}            (contraction 1 of r)
//   p_it.p_it = r.r + 2 beta r.p_{it-1} + beta^2 p_{it-1}.p_{it-1}
// with the three dot products left as block partials by the previous update.
// ---------------------------------------------------------------------------

// Loads the first partial of this thread (index threadIdx.x), clamped and
// unconditional, so that it can be issued early.
__device__ __forceinline__ double pload1(const double* a, int na) {
    return na > 0 ? a[min((int)threadIdx.x, na - 1)] : 0.0;
}

// CG head of iteration it: r.r, r.p_{it-1}, p_{it-1}.p_{it-1} from the
// partials (aux: three arrays of nbv), the stop rule (r.r <= tol^2 r0.r0,
// it >= maxiter, or non-finite), beta_it = r.r / r_{it-1}.r_{it-1} (0 at it =
// 0) and p_it.p_it.  Block 0 publishes them; every block takes the same
// decision.  The CG scalars the head reads are loaded when the kernel starts
// (earlier kernels wrote them; loading them there takes their latency off
// the end of the kernel).
struct HeadIn {
    int it, maxiter;
    double rr0, tol, rr_prev;
};
__device__ __forceinline__ HeadIn head_in(const CgScalars* sc) {
    HeadIn h;
    h.it = sc->it;
    h.maxiter = sc->maxiter;
    h.rr0 = sc->rr0;
    h.tol = sc->tol;
    h.rr_prev = sc->rr_prev;
    return h;
}

// CG head, part 1: this thread's share of the three partial sums (its
// pre-loaded first entries, then any further ones), reduced over the wave and
// parked in s3[q][wave]; the caller's barrier follows (it is shared with the
// contraction's own block reduction).
__device__ __forceinline__ void head_park(const double* aux, int nbv, int nth, double xa,
                                          double xb, double xc, double (*s3)[16]) {
    double t[3] = {0.0, 0.0, 0.0};
    if ((int)threadIdx.x < nbv) {
        t[0] = xa;
        t[1] = xb;
        t[2] = xc;
    }
    for (int i = nth + (int)threadIdx.x; i < nbv; i += nth) {
        t[0] += aux[i];
        t[1] += aux[nbv + i];
        t[2] += aux[2 * nbv + i];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double v = wave_sum(t[q]);
        if ((threadIdx.x & 63) == 0) s3[q][threadIdx.x >> 6] = v;
    }
}

// CG head, part 2 (after the barrier): the block sums r.r, r.p_old and
// p_old.p_old (waves in order, the same in every block), the stop test, beta
// and p.p; block 0 publishes them.  Returns false when CG stops.
__device__ __forceinline__ bool head_finish(const double (*s3)[16], int nw, const HeadIn& h,
                                            CgScalars* sc, double& beta) {
    double t[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double r = 0.0;
#pragma unroll
        for (int w = 0; w < 16; ++w)
            if (w < nw) r += s3[q][w];
        t[q] = r;
    }
    const double rr = t[0], rp = t[1], ppo = t[2];
    const int it = h.it;
    const double rr0 = it == 0 ? rr : h.rr0;  // (sc->rr0 is set by iteration 0's head)
    const double tol2 = h.tol * h.tol * rr0;
    const bool stop = !(rr > tol2) || it >= h.maxiter || !isfinite(rr);
    beta = it == 0 ? 0.0 : rr / h.rr_prev;
    const double pp = rr + 2.0 * beta * rp + beta * beta * ppo;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rr = rr;
        sc->iters = it;
        sc->beta = beta;
        sc->pp = pp;
        if (it == 0) {
            sc->rr0 = rr0;
            sc->tol2 = tol2;
        }
        if (stop) {
            sc->done = 1;
            if (!isfinite(rr)) sc->bad = 1;
        }
    }
    return !stop;
}

// block sum over nw <= 16 waves, identical order in every block (sh: 16 slots)
__device__ __forceinline__ double bsum_waves(double v, double* sh, int nw) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q)
        if (q < nw) r += sh[q];
    __syncthreads();
    return r;
}

// Waves per block and tiles per wave for `tiles` tiles over at most maxw waves.
static inline void wave_split(int tiles, int maxw, int& waves, int& per_wave) {
    per_wave = (tiles + maxw - 1) / maxw;
    waves = (tiles + per_wave - 1) / per_wave;
}

// ---------------------------------------------------------------------------
// contraction 1: w_k = t~_k . (P s~_k) for the 16 RT samples of a block.
// Wave w computes hidden tiles w, w + nw, ... (16 x 16 blocks of S P^T for
// each of the RT sample tiles, so each P fragment serves RT tiles) and
// weights them with tanh(theta).  Rows past n have zero spins (k_prep_spins),
// so their products vanish; their activation rows (the activation buffer
// holds whole blocks of rows) are read but only ever multiply those zeros.
// ---------------------------------------------------------------------------
constexpr int W5_RT = 2;        // FP64: sample tiles per block (32 samples)
constexpr int W_ROWS_MAX = 64;  // samples per contraction-1 block, largest form

// A load at a uniform base plus a 32-bit lane byte offset (the base stays in
// scalar registers, the lane part in one vector register).
template <typename T>
__device__ __forceinline__ T ld_at(const void* base, unsigned bytes) {
    return *(const T*)((const char*)base + bytes);
}

// FP64 operands of one 16-site group (sites g .. g + 15) of hidden tile ct:
// the residual rows g + 4 lk + e (e < 4) at column lr of the tile (global
// memory), and each sample tile's four spins at sites g + 4 lk .. + 3 (one
// 32-bit word of the block's spins, staged in LDS)
struct W5Src {
    const double* Pt;
    const double* Tb;      // the block's first activation row
    const uint32_t* Ls;    // the block's spins in LDS, LW words per sample row
    int Ma, Mw, LW;
    unsigned po, to, lo;   // lane offsets: residual and activations (bytes), spins (words)
};
template <int RT>
__device__ __forceinline__ void w5_group(const W5Src& c, int ct, int g, double (&b)[4],
                                         uint32_t (&s)[RT]) {
    const double* Pg = c.Pt + (size_t)g * c.Ma + 16 * ct;
#pragma unroll
    for (int e = 0; e < 4; ++e) b[e] = ld_at<double>(Pg + (size_t)e * c.Ma, c.po);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) s[rt] = c.Ls[c.lo + 16 * rt * c.LW + g / 4];
}
// the activations of hidden tile ct at the lane's accumulator rows (sample
// 16 rt + 4 q + lk of the block, hidden unit 16 ct + lr)
template <int RT>
__device__ __forceinline__ void w5_act(const W5Src& c, int ct, double (&t)[RT][4]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            t[rt][q] = ld_at<double>(c.Tb + (size_t)(16 * rt + 4 * q) * c.Mw + 16 * ct, c.to);
}
template <int RT>
__device__ __forceinline__ void w5_mfma(const double (&b)[4], const uint32_t (&s)[RT],
                                        v4d (&acc)[RT]) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const double a = (double)(int8_t)(s[rt] >> (8 * e));
            acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[e], acc[rt], 0, 0, 0);
        }
}
// the second group of a pair: its MFMAs, or, for the zero padding group past
// the last one (an odd number of groups), only a use of its operands, so that
// their loads stay where they were issued
__device__ __forceinline__ void w5_second(bool real, const double (&bq)[4],
                                          const uint32_t (&sq)[2], v4d (&acc)[2]) {
    if (real)
        w5_mfma<2>(bq, sq, acc);
    else
        asm volatile("" ::"v"(bq[0]), "v"(bq[1]), "v"(bq[2]), "v"(bq[3]), "v"(sq[0]), "v"(sq[1]));
}

// One hidden tile ct of a wave, its groups in pairs: the pair's second
// group loads (into bq) while the first group's MFMAs run, and the next
// pair's first group (into a; after the tile's last pair the first group of
// tile cn: the wave's next tile, or ct itself when there is none, so that
// every load is unconditional) while the second group's run.  The tile's
// activations are loaded with its first pair, ahead of its second group, and
// weight its 16 x 16 blocks into rs at the end.  Every wait then covers
// operands issued one group earlier.  ng groups in np = ceil(ng / 2) pairs.
template <int RT>
__device__ __forceinline__ void w5_tile(const W5Src& c, int ct, int cn, int ng, int np,
                                        double (&a)[4], uint32_t (&sa)[RT], double (&rs)[RT][4]) {
    v4d acc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc[rt] = v4d{0, 0, 0, 0};
    double tv[RT][4], bq[4];
    uint32_t sq[RT];
    w5_act<RT>(c, ct, tv);
    w5_group<RT>(c, ct, 16, bq, sq);
    __builtin_amdgcn_sched_barrier(0);  // loads ahead of the MFMAs that hide them
    w5_mfma<RT>(a, sa, acc);
    w5_group<RT>(c, np > 1 ? ct : cn, np > 1 ? 32 : 0, a, sa);
    __builtin_amdgcn_sched_barrier(0);
    w5_second(1 < ng, bq, sq, acc);
    for (int gp = 1; gp < np; ++gp) {
        w5_group<RT>(c, ct, 32 * gp + 16, bq, sq);
        __builtin_amdgcn_sched_barrier(0);
        w5_mfma<RT>(a, sa, acc);
        const bool more = gp + 1 < np;
        w5_group<RT>(c, more ? ct : cn, more ? 32 * (gp + 1) : 0, a, sa);
        __builtin_amdgcn_sched_barrier(0);
        w5_second(2 * gp + 1 < ng, bq, sq, acc);
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int q = 0; q < 4; ++q) rs[rt][q] += tv[rt][q] * acc[rt][q];
}

// FP64 path: at most 8 waves per block.  Sites run over the Na columns of the
// augmented layout (16 per group; the residual and Sp are zero past them,
// and a padding group completing the last pair only loads).  The block's
// spins (16 RT rows of Kb sites) are staged in LDS at the start, rows
// Kb + 8 bytes apart (lane quads of one row then fall in distinct banks).
__global__ __launch_bounds__(512) void k_w5(Dims d, const int8_t* __restrict__ Sp,
                                            const double* __restrict__ tact, long n,
                                            const double* __restrict__ Pt,
                                            double* __restrict__ w, double* __restrict__ wpart,
                                            const double* __restrict__ aux, int nbv,
                                            CgScalars* sc) {
    constexpr int RT = W5_RT;
    static_assert(RT == 2, "the keep-alives name two sample tiles");
    // the stop flag and the head's scalars; the flag is tested once the
    // first tile's loads are in flight
    const int done = sc->done;
    const HeadIn hin = head_in(sc);
    extern __shared__ uint32_t w5_spins[];
    __shared__ double wsh[16][16 * RT];
    __shared__ double wo[16 * RT];
    __shared__ double s3[3][16];
    const int tid = threadIdx.x, lane = tid & 63, nth = blockDim.x, nw = nth >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // tiles and their tests: scalar
    const int lr = lane & 15, lk = lane >> 4;
    const long r0 = (long)blockIdx.x * (16 * RT);
    // CG head inputs and the previous w, issued before the contraction
    const double xa = pload1(aux, nbv), xb = pload1(aux + nbv, nbv), xc = pload1(aux + 2 * nbv, nbv);
    const double wold = w[min(r0 + (lane & (16 * RT - 1)), n - 1)];
    // the block's spins: 16-byte pieces, the first two per thread issued now
    const int Kb = d.Kb, pr = Kb / 16, npc = 16 * RT * pr;
    uint4 sv[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int e = min(tid + u * nth, npc - 1);
        sv[u] = *(const uint4*)(Sp + (r0 + e / pr) * d.Kq + 16 * (e % pr));
    }
    const int nct = d.Ma / 16, ng = d.Na / 16, np = (ng + 1) / 2;
    W5Src c;
    c.Pt = Pt;
    c.Tb = tact + r0 * d.Mw;
    c.Ls = w5_spins;
    c.Ma = d.Ma;
    c.Mw = d.Mw;
    c.LW = (Kb + 8) / 4;
    c.po = 8u * (unsigned)(4 * lk * d.Ma + lr);
    c.to = 8u * (unsigned)(lk * d.Mw + lr);
    c.lo = (unsigned)(lr * c.LW + lk);
    double rs[RT][4], b[4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int q = 0; q < 4; ++q) rs[rt][q] = 0.0;
    // the first group's residual (every wave has at least one tile: wave_split)
    {
        const double* Pg = Pt + 16 * wave;
#pragma unroll
        for (int e = 0; e < 4; ++e) b[e] = ld_at<double>(Pg + (size_t)e * d.Ma, c.po);
    }
    asm volatile("" ::: "memory");  // the loads above go out before the stop test
    if (done) return;               // (uniform over the block, before any barrier)
    // the head's partials and the previous w go to LDS now (their loads were
    // issued first), so that they hold no registers through the contraction
    head_park(aux, nbv, nth, xa, xb, xc, s3);
    if (wave == 0 && lane < 16 * RT) wo[lane] = wold;
    auto put = [&](int e, const uint4& v) {
        uint2* q = (uint2*)(w5_spins + (e / pr) * c.LW + 4 * (e % pr));
        q[0] = make_uint2(v.x, v.y);
        q[1] = make_uint2(v.z, v.w);
    };
#pragma unroll
    for (int u = 0; u < 2; ++u)
        if (tid + u * nth < npc) put(tid + u * nth, sv[u]);
    for (int e = tid + 2 * nth; e < npc; e += nth)  // wide rows only
        put(e, *(const uint4*)(Sp + (r0 + e / pr) * d.Kq + 16 * (e % pr)));
    __syncthreads();
    uint32_t s[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) s[rt] = c.Ls[c.lo + 16 * rt * c.LW];
    for (int ct = wave; ct < nct; ct += nw)
        w5_tile<RT>(c, ct, ct + nw < nct ? ct + nw : ct, ng, np, b, s, rs);
    // the repeat loads issued with the last tile are used here, so that the
    // compiler keeps them ahead of that tile's matrix-core work (on the loop's
    // exit they would otherwise be dead and moved past it)
    asm volatile("" : "+v"(b[0]), "+v"(b[1]), "+v"(b[2]), "+v"(b[3]), "+v"(s[0]), "+v"(s[1]));
    // the sums over the 16 columns of the wave's tiles, parked in LDS behind
    // one barrier (shared with the head's)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double v = row16_sum(rs[rt][q]);
            if (lr == 0) wsh[wave][16 * rt + acc_row<double>(lk, q)] = v;
        }
    __syncthreads();
    double beta;
    if (!head_finish(s3, nw, hin, sc, beta)) return;
    if (wave == 0) {  // one lane per sample (waves in order), then over the block's samples
        double v = 0.0;
        const long k = r0 + lane;
        if (lane < 16 * RT) {
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (q < nw) v += wsh[q][lane];
            v += beta * wo[lane];  // J p = J r + beta J p_old
            if (k < n) w[k] = v;
        }
        const double t = wave_sum(lane < 16 * RT && k < n ? v : 0.0);
        if (lane == 0) wpart[blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// contraction 1, BF16 forms, 64 samples per block (four sample tiles).  Waves
// 0 .. nw - 2 take hidden tiles w, w + nw - 1, ...; the matrix cores compute
// the 16 x 16 blocks of P S^T with the hidden index as the row (A = the
// residual, two BF16 planes, B = the spins as FP4 codes converted to BF16),
// so that a lane holds four hidden rows of one sample: it weights them with
// that sample's activations and sums them in its own registers.  Both the
// residual and the activations are read in fragment order (pfrag_off,
// k_prep_tf).  The last wave runs the CG head meanwhile (the update's
// partials, stop test, beta) and after the barrier forms w = J r + beta w.
// ---------------------------------------------------------------------------
constexpr int W7_ROWS = 64;

// CG head from the three sums: stop test, beta and p.p; block 0 publishes.
// Returns false when CG stops.
__device__ __forceinline__ bool head_decide(double rr, double rp, double ppo, const HeadIn& h,
                                            CgScalars* sc, double& beta, bool lead_block) {
    const int it = h.it;
    const double rr0 = it == 0 ? rr : h.rr0;
    const double tol2 = h.tol * h.tol * rr0;
    const bool stop = !(rr > tol2) || it >= h.maxiter || !isfinite(rr);
    beta = it == 0 ? 0.0 : rr / h.rr_prev;
    const double pp = rr + 2.0 * beta * rp + beta * beta * ppo;
    if (lead_block && (threadIdx.x & 63) == 0) {
        sc->rr = rr;
        sc->iters = it;
        sc->beta = beta;
        sc->pp = pp;
        if (it == 0) {
            sc->rr0 = rr0;
            sc->tol2 = tol2;
        }
        if (stop) {
            sc->done = 1;
            if (!isfinite(rr)) sc->bad = 1;
        }
    }
    return !stop;
}

// (blk: the block's index within its run's grid)
__device__ __forceinline__ void w7_block(Dims d, const uint8_t* __restrict__ Sp,
                                         const float* __restrict__ Tf, long n,
                                         const uint16_t* __restrict__ Ph,
                                         double* __restrict__ w, double* __restrict__ wpart,
                                         const double* __restrict__ aux, int nbv, CgScalars* sc,
                                         int blk, int nwc) {
    constexpr int RT = W7_ROWS / 16;
    constexpr int HB = 4;  // head partials per lane issued up front, per sum
    // the stop flag; it is tested once the first loads are in flight
    const int done = sc->done;
    __shared__ double wsh[15][W7_ROWS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // waves 0 .. nwc - 1 take the hidden tiles, the last wave runs the head, and
    // any waves between them (a grouped launch sized for a larger run) idle
    const int nw = nwc, hw = (blockDim.x >> 6) - 1;
    const int lr = lane & 15, lk = lane >> 4;
    const long r0 = (long)blk * W7_ROWS;
    const int Kq = d.Kq, KB2 = d.Kq / 2, nct = d.Ma / 16, ng = d.Kq / 128;
    if (wave == hw) {
        // ---- the CG head: r.r, r.p_{it-1}, p_{it-1}.p_{it-1} from the update's
        // block partials (lane stride 64, then the wave: the same order in every block)
        const HeadIn hin = head_in(sc);
        double x[3][HB];
#pragma unroll
        for (int u = 0; u < HB; ++u) {
            const int i = 64 * u + lane;
#pragma unroll
            for (int k = 0; k < 3; ++k) x[k][u] = i < nbv ? aux[k * nbv + i] : 0.0;
        }
        const double wold = w[min(r0 + lane, n - 1)];
        asm volatile("" ::: "memory");  // the loads above go out before the stop test
        if (done) return;               // (uniform over the block, before any barrier)
        double t[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double a = 0.0;
#pragma unroll
            for (int u = 0; u < HB; ++u) a += x[k][u];
            for (int i = 64 * HB + lane; i < nbv; i += 64) a += aux[k * nbv + i];
            t[k] = wave_sum(a);
        }
        double beta;
        const bool go = head_decide(t[0], t[1], t[2], hin, sc, beta, blk == 0);
        __syncthreads();
        if (!go) return;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < 15; ++q)
            if (q < nw) v += wsh[q][lane];
        v += beta * wold;  // J p = J r + beta J p_old
        const long k = r0 + lane;
        if (k < n) w[k] = v;
        const double s = wave_sum(k < n ? v : 0.0);
        if (lane == 0) wpart[blk] = s;
        return;
    }
    if (wave >= nw) {  // an idle wave: the block's one barrier, or none once CG has stopped
        if (done) return;  // (uniform over the block, before any barrier)
        __syncthreads();
        return;
    }
    const uint16_t* Pl = Ph + (size_t)d.Ma * Kq;
    const uint8_t* sb = Sp + (r0 + lr) * KB2 + 16 * lk;  // sample tile rt: + 16 rt KB2
    float rs[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) rs[rt] = 0.0f;
    bool first = true;
    for (int ct = wave; ct < nct; ct += nw) {
        v4f acc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] = v4f{0, 0, 0, 0};
        float4 tv[RT];
        for (int g = 0; g < ng; ++g) {
            v8s bh[4], bl[4];
            uint4 sp[RT];  // 32 sites of the lane's sample in each tile, FP4
            const size_t po = (((size_t)ct * ng + g) * 4 * 64 + lane) * 8;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bh[u] = *(const v8s*)(Ph + po + 512 * u);
                bl[u] = *(const v8s*)(Pl + po + 512 * u);
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) sp[rt] = *(const uint4*)(sb + 16 * rt * KB2 + 64 * g);
            if (g == 0) {
                // the activations (needed after the MFMAs) behind the MFMA operands
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    tv[rt] = *(const float4*)(Tf + ((((size_t)blk * nct + ct) * RT + rt) * 64 + lane) * 4);
                if (first) {
                    asm volatile("" ::: "memory");  // the loads above go out before the stop test
                    if (done) return;               // (uniform over the block, before any barrier)
                    first = false;
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // the group's loads together
            // two sample tiles at a time: their hi products, then their lo products
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int rt = 0; rt < RT; rt += 2) {
                    const v8bf b0 = fp4x8_to_bf16(word_of(sp[rt], u));
                    const v8bf b1 = fp4x8_to_bf16(word_of(sp[rt + 1], u));
                    const v8bf ah = __builtin_bit_cast(v8bf, bh[u]), al = __builtin_bit_cast(v8bf, bl[u]);
                    acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b0, acc[rt], 0, 0, 0);
                    acc[rt + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b1, acc[rt + 1], 0, 0, 0);
                    acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b0, acc[rt], 0, 0, 0);
                    acc[rt + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b1, acc[rt + 1], 0, 0, 0);
                }
            }
        }
        // acc[rt][q]: hidden row ct 16 + 4 lk + q of sample 16 rt + lr
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
            rs[rt] += ((tv[rt].x * acc[rt][0] + tv[rt].y * acc[rt][1]) +
                       (tv[rt].z * acc[rt][2] + tv[rt].w * acc[rt][3]));
    }
    // each sample's rows summed over the four lane quads, parked for the head wave
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        float v = rs[rt];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (lk == 0) wsh[wave][16 * rt + lr] = (double)v;
    }
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_w7(Dims d, const uint8_t* __restrict__ Sp,
                                             const float* __restrict__ Tf, long n,
                                             const uint16_t* __restrict__ Ph,
                                             double* __restrict__ w, double* __restrict__ wpart,
                                             const double* __restrict__ aux, int nbv,
                                             CgScalars* sc) {
    w7_block(d, Sp, Tf, n, Ph, w, wpart, aux, nbv, sc, blockIdx.x, (blockDim.x >> 6) - 1);
}

// ---------------------------------------------------------------------------
// contraction 2: part[q][j][i] = sum_{k in range q} t~_kj z_k s~_ki
// v_mode 0: z_k = (w_k - mean w) / n with mean w from the contraction-1
// partials, and the blocks of hidden tile 0 write their range's partial of
// p . G p without the shift (sum_k z_k (w_k - mean w)); v_mode 1: z_k = v_k.
// Block order: the hardware deals consecutive blocks to the 8 XCDs in turn;
// the blocks of one sample range (or chunk) are placed on one XCD where the
// grid allows, so that its spins are brought into a single L2.
// ---------------------------------------------------------------------------
constexpr int NXCD = 8;
// BF16 forms: one block per (hidden tile, chunk of 512 samples); BF16 rows
// 520 halves apart
constexpr int O16_KC = 512, O16_KP = O16_KC + 8;

// block -> (hidden tile, chunk), chunks grouped by XCD
__device__ __forceinline__ void outer_block(int L, int nj, int& jt, int& kc) {
    const int x = L % NXCD, m = L / NXCD;
    jt = m % nj;
    kc = x + NXCD * (m / nj);
}

// FP64 path.  Block (pass, jt, q): hidden tile jt, the site tiles of the
// pass (up to 32; PT per active wave, the active waves taking tiles w,
// w + nwa, ...), and the q-th of ks near-equal ranges of 16-sample units (ks
// chosen so that the blocks fill the CUs in one round, all with the same
// work: two 512-thread blocks or one 1024-thread block per CU).
// The range streams through LDS in sub-chunks of SC samples (64 in 512-thread
// blocks, 128 in 1,024-thread blocks: every thread stages at least one 16-byte
// unit; shorter sub-chunks start the matrix cores sooner): while the matrix
// cores take a = t~ z of the current sub-chunk from LDS, the next sub-chunk's
// t~ and z source and the spins are loaded; every wave keeps the sums of its
// site tiles in registers over the whole range.  The FP64 MFMA takes A = a and
// B = the int8 spins as +1 / -1 (0 on padding sites); within 16 samples,
// k-step e of lane quad lk takes sample 4 lk + e.
template <int SC>
struct O9 {
    static constexpr int LD = SC + 1;       // doubles between staged rows (odd)
    static constexpr int NU = SC / 16;      // 16-sample units per sub-chunk
    static constexpr int PR = SC / 2;       // 16-byte staging units (sample pairs) per row
    static constexpr int PIECES = 16 * PR;  // 16-byte staging units of a sub-chunk
};

struct O9Range {
    long k0, k1;  // the block's samples [k0, k1)
    int nsc;      // sub-chunks
};

// t~ and the z source of sub-chunk c (16-byte units: thread unit e is row
// e / O9<SC>::PR, samples 2 (e % O9<SC>::PR) + {0, 1}), clamped into the block's range
template <int SC, int NTH>
__device__ __forceinline__ void o9_load(const double* __restrict__ Tj, const double* __restrict__ v,
                                        long Nsp, const O9Range& R, int c,
                                        double2 (&ta)[O9<SC>::PIECES / NTH],
                                        double2 (&va)[O9<SC>::PIECES / NTH]) {
#pragma unroll
    for (int i = 0; i < O9<SC>::PIECES / NTH; ++i) {
        const int e = threadIdx.x + NTH * i;
        const long k = min(R.k0 + (long)c * SC + 2 * (e % O9<SC>::PR), R.k1 - 2);
        ta[i] = *(const double2*)(Tj + (size_t)(e / O9<SC>::PR) * Nsp + k);
        va[i] = *(const double2*)(v + k);
    }
}
// a = t~ z of sub-chunk c into LDS (zero past the range and past n); the
// threads holding row 0 add up z_k (v_k - shift) (the p . G p partial)
template <int SC, int NTH>
__device__ __forceinline__ void o9_stage(double* __restrict__ A, const O9Range& R, int c, long n,
                                         double shift, double scale,
                                         const double2 (&ta)[O9<SC>::PIECES / NTH],
                                         const double2 (&va)[O9<SC>::PIECES / NTH], double& zw) {
#pragma unroll
    for (int i = 0; i < O9<SC>::PIECES / NTH; ++i) {
        const int e = threadIdx.x + NTH * i;
        const int r = e / O9<SC>::PR, c2 = 2 * (e % O9<SC>::PR);
        const long k = R.k0 + (long)c * SC + c2;
        const bool ok0 = k < R.k1 && k < n, ok1 = k + 1 < R.k1 && k + 1 < n;
        const double z0 = ok0 ? (va[i].x - shift) * scale : 0.0;
        const double z1 = ok1 ? (va[i].y - shift) * scale : 0.0;
        A[r * O9<SC>::LD + c2] = ta[i].x * z0;
        A[r * O9<SC>::LD + c2 + 1] = ta[i].y * z1;
        if (r == 0) zw += z0 * (va[i].x - shift) + z1 * (va[i].y - shift);
    }
}
// the spins of site tile it for sub-chunk c: one word (4 samples) per unit
template <int SC, int PT>
__device__ __forceinline__ void o9_spins(const int8_t* __restrict__ St, long Nsp, const O9Range& R,
                                         int c, const int (&its)[PT], int lr, int lk,
                                         uint32_t (&sb)[PT][O9<SC>::NU]) {
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int u = 0; u < O9<SC>::NU; ++u) {
            const long k = min(R.k0 + (long)c * SC + 16 * u, R.k1 - 16) + 4 * lk;
            sb[p][u] = *(const uint32_t*)(St + (size_t)(its[p] * 16 + lr) * Nsp + k);
        }
}

// the MFMAs of one sub-chunk for the wave's first NT site tiles: units of 16
// samples (those past the range: none), the LDS operands of unit u + 1 read
// while unit u's MFMAs run
template <int SC, int NT, int PT, int CH>
__device__ __forceinline__ void o9_units(const double* __restrict__ A, int nu,
                                         const uint32_t (&sb)[PT][O9<SC>::NU], v4d (&acc)[PT][CH]) {
    double a[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) a[e] = A[e];
#pragma unroll
    for (int u = 0; u < O9<SC>::NU; ++u) {
        double an[4];
        if (u + 1 < O9<SC>::NU) {
#pragma unroll
            for (int e = 0; e < 4; ++e) an[e] = A[16 * (u + 1) + e];
        }
        if (u < nu) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int p = 0; p < NT; ++p) {
                    const double b = (double)(int8_t)(sb[p][u] >> (8 * e));
                    acc[p][e % CH] =
                        __builtin_amdgcn_mfma_f64_16x16x4f64(a[e], b, acc[p][e % CH], 0, 0, 0);
                }
        }
        if (u + 1 < O9<SC>::NU) {
#pragma unroll
            for (int e = 0; e < 4; ++e) a[e] = an[e];
        }
        __builtin_amdgcn_sched_barrier(0);  // one unit's LDS operands in flight at a time
    }
}

template <int PT, int NTH>
__global__ __launch_bounds__(NTH) void k_outer9(Dims d, const int8_t* __restrict__ St,
                                                const double* __restrict__ Th, long Nsp, long n,
                                                const double* __restrict__ v, int v_mode,
                                                const double* __restrict__ wpart, int nbw,
                                                double* __restrict__ part, int ks, int tpp,
                                                int nwa, double* __restrict__ papart,
                                                const CgScalars* __restrict__ sc) {
    constexpr int SC = NTH == 512 ? 64 : 128;  // samples per sub-chunk
    constexpr int UT = O9<SC>::PIECES / NTH;  // staging units per thread
    // stop flag of the CG product, tested once the block's loads are in flight
    const int done = v_mode == 0 ? sc->done : 0;
    constexpr int CH = PT == 1 ? 4 : 1;  // accumulation chains per site tile
    constexpr int BW = 2;                // mean-w partials per thread issued up front
    __shared__ double As[2][16 * O9<SC>::LD];
    __shared__ double sh[16];
    const int nj = d.Ma / 16, ni = d.Na / 16;
    // work item (pass, q, jt), range-major, from the block index: XCD x (the
    // blocks x, x + 8, ...) takes a contiguous run of items, so that the
    // blocks of one range share one or two L2s
    const int nit = (int)gridDim.x, L = blockIdx.x, x = L % NXCD;
    const int before = x * (nit / NXCD) + min(x, nit % NXCD);  // items of XCDs 0 .. x - 1
    const int item = before + L / NXCD;
    const int pass = item / (nj * ks), i2 = item - pass * nj * ks;
    const int q = i2 / nj, jt = i2 - q * nj;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    const long U = (n + 15) / 16;
    O9Range R;
    R.k0 = 16 * ((long)q * U / ks);
    R.k1 = 16 * (((long)q + 1) * U / ks);
    R.nsc = (int)((R.k1 - R.k0 + SC - 1) / SC);
    // this wave's site tiles (clamped to a valid one; nact of them count)
    const int t0 = pass * tpp, t1 = min(ni, t0 + tpp);
    int its[PT], nact = 0;
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        const int it = wave < nwa ? t0 + wave + nwa * p : t1;
        nact += it < t1 ? 1 : 0;
        its[p] = it < t1 ? it : t1 - 1;
    }
    const double* Tj = Th + (size_t)jt * 16 * Nsp;
    // ---- issue: mean-w partials, the first sub-chunk and its spins
    double wp[BW];
#pragma unroll
    for (int u = 0; u < BW; ++u) {
        const int b = u * NTH + tid;
        wp[u] = (v_mode == 0 && b < nbw) ? wpart[b] : 0.0;
    }
    double2 ta[UT], va[UT];
    o9_load<SC, NTH>(Tj, v, Nsp, R, 0, ta, va);
    uint32_t sb[PT][O9<SC>::NU];
    o9_spins<SC, PT>(St, Nsp, R, 0, its, lr, lk, sb);
    asm volatile("" ::: "memory");  // the loads above go out before the stop test
    if (done) return;               // (uniform over the block, before any barrier)
    double shift = 0.0, scale = 1.0;
    if (v_mode == 0) {
        double a = 0.0;
#pragma unroll
        for (int u = 0; u < BW; ++u) a += wp[u];
        for (int b = BW * NTH + tid; b < nbw; b += NTH) a += wpart[b];
        shift = bsum_waves(a, sh, NTH / 64) / (double)n;
        scale = 1.0 / (double)n;
    }
    double zw = 0.0;
    o9_stage<SC, NTH>(As[0], R, 0, n, shift, scale, ta, va, zw);
    __syncthreads();
    v4d acc[PT][CH];
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int h = 0; h < CH; ++h) acc[p][h] = v4d{0, 0, 0, 0};
    for (int c = 0; c < R.nsc; ++c) {
        // the next sub-chunk (this one again after the last: every load unconditional)
        const int cn = c + 1 < R.nsc ? c + 1 : c;
        o9_load<SC, NTH>(Tj, v, Nsp, R, cn, ta, va);
        uint32_t sn[PT][O9<SC>::NU];
        o9_spins<SC, PT>(St, Nsp, R, cn, its, lr, lk, sn);
        __builtin_amdgcn_sched_barrier(0);  // those loads ahead of the MFMAs that hide them
        const double* A = As[c & 1] + lr * O9<SC>::LD + 4 * lk;
        const int nu = (int)min((long)O9<SC>::NU, (R.k1 - R.k0) / 16 - (long)c * O9<SC>::NU);
        if (nact == PT)
            o9_units<SC, PT, PT, CH>(A, nu, sb, acc);
        else if (nact > 0)
            o9_units<SC, 1, PT, CH>(A, nu, sb, acc);
        if (c + 1 < R.nsc) {
            o9_stage<SC, NTH>(As[(c + 1) & 1], R, c + 1, n, shift, scale, ta, va, zw);
        } else {  // a use of the repeat loads, which keeps them where they were issued
#pragma unroll
            for (int i = 0; i < UT; ++i) asm volatile("" ::"v"(ta[i].x), "v"(va[i].x));
        }
#pragma unroll
        for (int p = 0; p < PT; ++p)
#pragma unroll
            for (int u = 0; u < O9<SC>::NU; ++u) sb[p][u] = sn[p][u];
        __syncthreads();
    }
    // p . G p = sum_k z_k (w_k - mean w) (G p = J^T z, w = J p): one partial per
    // range, from the blocks of hidden tile 0
    if (v_mode == 0 && jt == 0 && pass == 0) {
        const double t = bsum_waves(zw, sh, NTH / 64);
        if (tid == 0) papart[q] = t;
    }
    double* out = part + (size_t)q * d.Ma * d.Na;
#pragma unroll
    for (int p = 0; p < PT; ++p)
        if (p < nact) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double t;
                if constexpr (CH == 4)
                    t = (acc[p][0][r] + acc[p][1][r]) + (acc[p][2][r] + acc[p][3][r]);
                else
                    t = acc[p][0][r];
                out[(size_t)(jt * 16 + acc_row<double>(lk, r)) * d.Na + its[p] * 16 + lr] = t;
            }
        }
}

// BF16 forms: t~ (FP32, [Ma][Nsp]) is scaled by z while it is staged: the
// LDS tile holds a_kj = t~_kj z_k (FP32 product) as two BF16 terms hi + lo
// (hardware round-to-nearest conversion), and B is the spin matrix itself,
// +1 / -1, exact in BF16 (FP4 codes, converted two per instruction).  Two
// MFMAs per k-step (hi and lo) with FP32 accumulation; the error of a
// product is that of the two-term split of a, about 2^-17 relative.
// 512 threads: for the staging, thread t takes samples 4 (t % 128) .. + 3 of
// rows 4 (t / 128) .. + 3 and forms their z itself (every wave sums the mean
// of w in the same order, so no barrier precedes the staging); for the
// contraction, wave w takes site tiles w, w + 8, ...
constexpr int O8_THREADS = 512;
// (blk: the block's index within its run's grid)
__device__ __forceinline__ void outer8_block(Dims d, const uint8_t* __restrict__ St,
                                             const float* __restrict__ Th, long Nsp, long n,
                                             const double* __restrict__ v, int v_mode,
                                             const double* __restrict__ wpart, int nbw,
                                             float* __restrict__ part, int ksplit,
                                             double* __restrict__ papart,
                                             const CgScalars* __restrict__ sc, int blk) {
    // stop flag of the CG product, tested once the block's loads are in flight
    const int done = v_mode == 0 ? sc->done : 0;
    constexpr int KC = O16_KC, KP = O16_KP;
    constexpr int NW = O8_THREADS / 64;
    __shared__ __align__(16) uint16_t As[2 * 16 * KP];  // hi rows, then lo rows
    __shared__ double sh[NW];
    const int nj = d.Ma / 16;
    int jt, kc;
    outer_block(blk, nj, jt, kc);
    if (kc >= ksplit) return;  // no chunk for this block
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long kbeg = (long)kc * KC;
    const int nit = d.Na / 16;
    const int c = tid & 127, rg = tid >> 7;  // staging: samples 4 c.., rows 4 rg..
    // ---- issue: t~ rows, the four samples' v, mean-w partials (wave 0), spins
    const float* Ab = Th + (size_t)(jt * 16 + 4 * rg) * Nsp + kbeg + 4 * c;
    float4 ta[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) ta[q] = *(const float4*)(Ab + (size_t)q * Nsp);
    const double2 v01 = *(const double2*)(v + kbeg + 4 * c);  // v has Nsp slots
    const double2 v23 = *(const double2*)(v + kbeg + 4 * c + 2);
    const double vk[4] = {v01.x, v01.y, v23.x, v23.y};
    double wp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int b = 64 * u + lane;
        wp[u] = (v_mode == 0 && b < nbw) ? wpart[b] : 0.0;
    }
    uint4 sp[4];  // FP4 spins of the lane's site in the chunk, positions 128 lk ..
    auto load_spins = [&](int it) {
        const uint8_t* Sr = St + (size_t)(it * 16 + lr) * (Nsp / 2) + kbeg / 2 + 64 * lk;
#pragma unroll
        for (int q = 0; q < 4; ++q) sp[q] = *(const uint4*)(Sr + 16 * q);
    };
    if (wave < nit) load_spins(wave);
    asm volatile("" ::: "memory");  // the loads above go out before the stop test
    if (done) return;               // (uniform over the block, before any barrier)
    __builtin_amdgcn_sched_barrier(0);  // all of the above in flight before any use
    // ---- mean w over the batch, summed by every wave in the same fixed order
    double shift = 0.0, scale = 1.0;
    if (v_mode == 0) {
        double a = (wp[0] + wp[1]) + (wp[2] + wp[3]);
        for (int b = 256 + lane; b < nbw; b += 64) a += wpart[b];
        shift = wave_sum(a) / (double)n;
        scale = 1.0 / (double)n;
    }
    float z[4];
    double zw = 0.0;  // this thread's part of sum_k z_k (w_k - mean w) (row group 0)
#pragma unroll
    for (int e = 0; e < 4; ++e) {  // (v past n is not read as a number)
        const bool in = kbeg + 4 * c + e < n;
        const double zz = in ? (vk[e] - shift) * scale : 0.0;
        zw += in ? zz * (vk[e] - shift) : 0.0;
        z[e] = (float)zz;
    }
    // ---- stage a = t~ z as hi / lo BF16 rows
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t h0, l0, h1, l1;
        split_pk(ta[q].x * z[0], ta[q].y * z[1], h0, l0);
        split_pk(ta[q].z * z[2], ta[q].w * z[3], h1, l1);
        const int row = 4 * rg + q;
        *(uint2*)(As + row * KP + 4 * c) = make_uint2(h0, h1);
        *(uint2*)(As + (16 + row) * KP + 4 * c) = make_uint2(l0, l1);
    }
    // p . G p = sum_k z_k (w_k - mean w) (G p = J^T z, w = J p): one partial per
    // chunk, from the blocks of hidden tile 0 (row group 0 = waves 0 and 1)
    const bool pgp = v_mode == 0 && jt == 0;
    if (pgp && rg == 0) {
        zw = wave_sum(zw);
        if (lane == 0) sh[wave] = zw;
    }
    __syncthreads();
    if (pgp && tid == 0) papart[kc] = sh[0] + sh[1];
    for (int it = wave; it < nit; it += NW) {
        if (it != wave) load_spins(it);
        v4f acc = v4f{0, 0, 0, 0}, acc2 = v4f{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < KC / 32; ++u) {
            const int kk = 32 * u + 8 * lk;
            const v8bf ah = __builtin_bit_cast(v8bf, *(const v8s*)(As + lr * KP + kk));
            const v8bf al = __builtin_bit_cast(v8bf, *(const v8s*)(As + (16 + lr) * KP + kk));
            const v8bf b = fp4x8_to_bf16(word_of(sp[u >> 2], u & 3));
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b, acc, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b, acc2, 0, 0, 0);
            if ((u & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // four k-steps of operands live at a time
        }
        float* out = part + (size_t)kc * d.Ma * d.Na;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            out[(size_t)(jt * 16 + acc_row<float>(lk, q)) * d.Na + it * 16 + lr] = acc[q] + acc2[q];
    }
}

__global__ __launch_bounds__(O8_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_outer8(Dims d, const uint8_t* __restrict__ St,
                                                       const float* __restrict__ Th, long Nsp, long n,
                                                       const double* __restrict__ v, int v_mode,
                                                       const double* __restrict__ wpart, int nbw,
                                                       float* __restrict__ part, int ksplit,
                                                       double* __restrict__ papart,
                                                       const CgScalars* __restrict__ sc) {
    outer8_block(d, St, Th, Nsp, n, v, v_mode, wpart, nbw, part, ksplit, papart, sc, blockIdx.x);
}

// out[e] = sum_kc part[kc][e] + shift p[e] (parameter entries only); with p,
// also the block partials of p . out.  A block covers 64 entries; wave w sums
// the chunk slabs [w ks/4, (w + 1) ks/4) and the four sums meet in LDS.
template <typename R>
__global__ __launch_bounds__(256) void k_reduce3(Dims d, const R* __restrict__ part, int ksplit,
                                                 const double* __restrict__ p, double shift,
                                                 double* __restrict__ out,
                                                 double* __restrict__ pap,
                                                 const CgScalars* __restrict__ sc, int cg) {
    if (cg && sc->done) return;
    __shared__ double ws[4][64];
    __shared__ double sh[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int total = d.Ma * d.Na;
    const int e = blockIdx.x * 64 + lane;
    const int ec = e < total ? e : total - 1;
    const int kb = wave * ksplit / 4, ke = (wave + 1) * ksplit / 4;
    double val = 0.0;
    int kc = kb;
    for (; kc + 16 <= ke; kc += 16) {
        R x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) x[u] = part[(size_t)(kc + u) * total + ec];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 16; ++u) val += (double)x[u];
    }
    for (; kc < ke; ++kc) val += (double)part[(size_t)kc * total + ec];
    ws[wave][lane] = val;
    __syncthreads();
    double dot = 0.0;
    if (wave == 0 && e < total) {
        const int j = e / d.Na, i = e - j * d.Na;
        const bool keep = (j < d.M && i < d.N) || (d.hb && j < d.M && i == d.N) ||
                          (d.vb && j == d.M && i < d.N);
        double o = 0.0;
        if (keep) {
            o = (ws[0][lane] + ws[1][lane]) + (ws[2][lane] + ws[3][lane]);
            if (p) o += shift * p[e];
        }
        out[e] = o;
        if (p) dot = o * p[e];
    }
    if (!cg) return;
    dot = bsum256(dot, sh);
    if (threadIdx.x == 0) pap[blockIdx.x] = dot;
}

// CG update of iteration it (FP64 path), 64 entries per block (wave w sums chunk slabs
// [w ks/4, (w+1) ks/4); after one barrier wave 0 finishes alone), with r.r,
// beta and p.p from the head:
//   p_it = r + beta p_{it-1};  Ap = sum_kc part[kc] + shift p_it (parameter
//   entries only);  p.Ap = sum of the per-chunk partials of p.G p + shift p.p;
//   alpha = r.r / p.Ap;  x += alpha p_it;  r -= alpha Ap;
// writes p_it, r (also in the contraction-1 operand layout) and the block
// partials of r.r, r.p_it, p_it.p_it for the next head.  Block 0 advances the
// iteration index and, when given a pinned host word, stores the stop flag
// there (the last update of a batch of iterations does).
// SW: slot slabs per wave loaded up front (at least ceil(ksplit / 4) where that
// is at most 16; further slabs are read in the loop that follows)
template <int SW>
__global__ __launch_bounds__(256) void k_update4(Dims d, const double* part, int ksplit, double* x,
                                                 double* r, const double* p_old, double* p_new,
                                                 void* Rop, const double* papart, int npa,
                                                 double* aux_next, int nbv, CgScalars* sc,
                                                 volatile int32_t* host_flag) {
    __shared__ double ws[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int total = d.Ma * d.Na;
    const int e = blockIdx.x * 64 + lane;
    const int ec = e < total ? e : total - 1;
    // every load that does not depend on the scalars, issued up front
    const int kb = wave * ksplit / 4, ke = (wave + 1) * ksplit / 4;
    double xs[SW];
#pragma unroll
    for (int u = 0; u < SW; ++u) xs[u] = part[(size_t)min(kb + u, ksplit - 1) * total + ec];
    const double xe = x[ec], re0 = r[ec], po = p_old[ec];
    double xa[4];  // p.Gp chunk partials lane, lane + 64, ... (summed by wave 0)
#pragma unroll
    for (int u = 0; u < 4; ++u) xa[u] = npa > 0 ? papart[min(u * 64 + lane, npa - 1)] : 0.0;
    // the CG scalars with the stop flag (one round trip)
    const int done = sc->done;
    const double shift = sc->shift, rr = sc->rr, beta = sc->beta, pp = sc->pp;
    asm volatile("" ::: "memory");  // keep the loads above ahead of the stop test
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (done) {
        if (host_flag && lead) *host_flag = 1;
        return;
    }
    double val = 0.0;
#pragma unroll
    for (int u = 0; u < SW; ++u)
        if (kb + u < ke) val += (double)xs[u];
    for (int kc = kb + SW; kc < ke; ++kc) val += (double)part[(size_t)kc * total + ec];
    ws[wave][lane] = val;
    __syncthreads();
    if (wave != 0) return;  // waves 1-3 only summed chunk slabs
    // p.G p: the chunk partials in a fixed order (the same in every block)
    double tg = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (u * 64 + lane < npa) tg += xa[u];
    for (int c = 256 + lane; c < npa; c += 64) tg += papart[c];
    const double pGp = wave_sum(tg);
    const double pAp = pGp + shift * pp;
    const double alpha = rr / pAp;
    if (!(pAp > 0.0) || !isfinite(alpha)) {
        if (lead) {
            sc->bad = 1;
            sc->done = 1;
            if (host_flag) *host_flag = 1;
        }
        return;
    }
    if (lead) {
        sc->alpha = alpha;
        sc->pAp = pAp;
        sc->rr_prev = rr;
        sc->it += 1;  // read by the next head
        if (host_flag) *host_flag = 0;
    }
    double q[3] = {0.0, 0.0, 0.0};
    if (e < total) {
        const int j = e / d.Na, i = e - j * d.Na;
        const bool keep = (j < d.M && i < d.N) || (d.hb && j < d.M && i == d.N) ||
                          (d.vb && j == d.M && i < d.N);
        const double pn = re0 + beta * po;
        const double ap = keep ? (ws[0][lane] + ws[1][lane]) + (ws[2][lane] + ws[3][lane]) + shift * pn
                               : 0.0;
        const double rn = re0 - alpha * ap;
        x[e] = xe + alpha * pn;
        r[e] = rn;
        p_new[e] = pn;
        ((double*)Rop)[(size_t)i * d.Ma + j] = rn;
        q[0] = rn * rn;
        q[1] = rn * pn;
        q[2] = pn * pn;
    }
    // the block's partials of r.r, r.p and p.p for the next head
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = wave_sum(q[k]);
        if (lane == 0) aux_next[(size_t)k * nbv + blockIdx.x] = v;
    }
}

// BF16 forms: the CG update as above with 128 entries per block, two per
// lane (FP32 chunk partial pairs; FP64 vectors as pairs), the residual
// written to the contraction-1 operand as its two BF16 terms in fragment
// order (pfrag_off).
// (blk: the block's index within its run's grid; SW as for k_update4)
template <int SW>
__device__ __forceinline__ void update5_block(Dims d, const float* part, int ksplit, double* x,
                                              double* r, const double* p_old, double* p_new,
                                              uint16_t* Rop, const double* papart, int npa,
                                              double* aux_next, int nbv, CgScalars* sc,
                                              volatile int32_t* host_flag, int blk) {
    __shared__ double2 ws[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int total = d.Ma * d.Na;  // even (Na is a multiple of 16)
    const int e = blk * 128 + 2 * lane;
    const int ec = e < total ? e : total - 2;
    // every load that does not depend on the scalars, issued up front
    const int kb = wave * ksplit / 4, ke = (wave + 1) * ksplit / 4;
    float2 xs[SW];
#pragma unroll
    for (int u = 0; u < SW; ++u)
        xs[u] = *(const float2*)(part + (size_t)min(kb + u, ksplit - 1) * total + ec);
    const double2 xe = *(const double2*)(x + ec), re0 = *(const double2*)(r + ec),
                  po = *(const double2*)(p_old + ec);
    double xa[4];  // p.Gp chunk partials lane, lane + 64, ... (summed by wave 0)
#pragma unroll
    for (int u = 0; u < 4; ++u) xa[u] = npa > 0 ? papart[min(u * 64 + lane, npa - 1)] : 0.0;
    // the CG scalars with the stop flag (one round trip)
    const int done = sc->done;
    const double shift = sc->shift, rr = sc->rr, beta = sc->beta, pp = sc->pp;
    asm volatile("" ::: "memory");  // keep the loads above ahead of the stop test
    const bool lead = blk == 0 && threadIdx.x == 0;
    if (done) {
        if (host_flag && lead) *host_flag = 1;
        return;
    }
    double v0 = 0.0, v1 = 0.0;
#pragma unroll
    for (int u = 0; u < SW; ++u)
        if (kb + u < ke) {
            v0 += (double)xs[u].x;
            v1 += (double)xs[u].y;
        }
    for (int kc = kb + SW; kc < ke; ++kc) {
        const float2 t = *(const float2*)(part + (size_t)kc * total + ec);
        v0 += (double)t.x;
        v1 += (double)t.y;
    }
    ws[wave][lane] = make_double2(v0, v1);
    __syncthreads();
    if (wave != 0) return;  // waves 1-3 only summed chunk slabs
    // p.G p: the chunk partials in a fixed order (the same in every block)
    double tg = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (u * 64 + lane < npa) tg += xa[u];
    for (int c = 256 + lane; c < npa; c += 64) tg += papart[c];
    const double pGp = wave_sum(tg);
    const double pAp = pGp + shift * pp;
    const double alpha = rr / pAp;
    if (!(pAp > 0.0) || !isfinite(alpha)) {
        if (lead) {
            sc->bad = 1;
            sc->done = 1;
            if (host_flag) *host_flag = 1;
        }
        return;
    }
    if (lead) {
        sc->alpha = alpha;
        sc->pAp = pAp;
        sc->rr_prev = rr;
        sc->it += 1;  // read by the next head
        if (host_flag) *host_flag = 0;
    }
    double q[3] = {0.0, 0.0, 0.0};
    if (e < total) {
        const int j = e / d.Na, i = e - j * d.Na;  // entries (j, i) and (j, i + 1)
        auto keep = [&](int ii) {
            return (j < d.M && ii < d.N) || (d.hb && j < d.M && ii == d.N) ||
                   (d.vb && j == d.M && ii < d.N);
        };
        const bool k0 = keep(i), k1 = keep(i + 1);
        const double2 s0 = ws[0][lane], s1 = ws[1][lane], s2 = ws[2][lane], s3 = ws[3][lane];
        const double pn0 = re0.x + beta * po.x, pn1 = re0.y + beta * po.y;
        const double ap0 = k0 ? (s0.x + s1.x) + (s2.x + s3.x) + shift * pn0 : 0.0;
        const double ap1 = k1 ? (s0.y + s1.y) + (s2.y + s3.y) + shift * pn1 : 0.0;
        const double rn0 = re0.x - alpha * ap0, rn1 = re0.y - alpha * ap1;
        *(double2*)(x + e) = make_double2(xe.x + alpha * pn0, xe.y + alpha * pn1);
        *(double2*)(r + e) = make_double2(rn0, rn1);
        *(double2*)(p_new + e) = make_double2(pn0, pn1);
        uint32_t hi, lo;
        split_pk((float)rn0, (float)rn1, hi, lo);
        const size_t o = pfrag_off(j, i, d.Kq / 128);
        *(uint32_t*)(Rop + o) = hi;
        *(uint32_t*)(Rop + (size_t)d.Ma * d.Kq + o) = lo;
        q[0] = rn0 * rn0 + rn1 * rn1;
        q[1] = rn0 * pn0 + rn1 * pn1;
        q[2] = pn0 * pn0 + pn1 * pn1;
    }
    // the block's partials of r.r, r.p and p.p for the next head
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = wave_sum(q[k]);
        if (lane == 0) aux_next[(size_t)k * nbv + blk] = v;
    }
}

template <int SW>
__global__ __launch_bounds__(256) void k_update5(Dims d, const float* part, int ksplit, double* x,
                                                 double* r, const double* p_old, double* p_new,
                                                 uint16_t* Rop, const double* papart, int npa,
                                                 double* aux_next, int nbv, CgScalars* sc,
                                                 volatile int32_t* host_flag) {
    update5_block<SW>(d, part, ksplit, x, r, p_old, p_new, Rop, papart, npa, aux_next, nbv, sc,
                      host_flag, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Grouped CG iterations (BF16 forms): one launch of a kernel class runs the
// blocks of several independent runs.  Block b of a launch belongs to the run
// r with first[r] <= b < first[r + 1] and runs as block b - first[r] of that
// run's own launch, on that run's operands (table entry r): every run keeps
// its own blocks and its own fixed-order sums.  Contraction-2 block counts
// are multiples of 8, so every run's blocks keep their XCD placement.  The
// contraction-1 launches (one per block size) number their blocks on from
// one another (base: the launch's first block).
// ---------------------------------------------------------------------------
// the run of block b (first[] ascending, padded with INT_MAX past the last
// run; every entry is read, so the reads go out together)
__device__ __forceinline__ int group_run(const int* __restrict__ first, int b) {
    int r = 0;
#pragma unroll
    for (int i = 1; i < CG_GROUP_MAX; ++i) r += first[i] <= b ? 1 : 0;
    return r;
}

__global__ __launch_bounds__(1024) void k_w7_group(const CgGroupTable* __restrict__ t, int base,
                                                   int par) {
    const int b = base + (int)blockIdx.x;
    const int r = group_run(t->first_w, b);
    const CgGroupRun& R = t->run[r];
    w7_block(R.d, (const uint8_t*)R.Sp, R.Tf, R.n, (const uint16_t*)R.Rop, R.w, R.wpart,
             R.aux + (size_t)par * 3 * R.nbv, R.nbv, R.sc, b - t->first_w[r], R.nwc);
}

__global__ __launch_bounds__(O8_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_outer8_group(
    const CgGroupTable* __restrict__ t) {
    const int r = group_run(t->first_o, blockIdx.x);
    const CgGroupRun& R = t->run[r];
    outer8_block(R.d, (const uint8_t*)R.St, (const float*)R.Th, R.Nsp, R.n, R.w, 0, R.wpart,
                 R.nbw, (float*)R.part, R.ks, R.papart, R.sc, blockIdx.x - t->first_o[r]);
}

template <int SW>
__global__ __launch_bounds__(256) void k_update5_group(const CgGroupTable* __restrict__ t, int par,
                                                       int write_flag) {
    const int r = group_run(t->first_u, blockIdx.x);
    const CgGroupRun& R = t->run[r];
    update5_block<SW>(R.d, (const float*)R.part, R.ks, R.x, R.r, par ? R.p2 : R.p, par ? R.p : R.p2,
                  (uint16_t*)R.Rop, R.papart, R.ks, R.aux + (size_t)(par ^ 1) * 3 * R.nbv, R.nbv,
                  R.sc, write_flag ? R.host_flag : nullptr, blockIdx.x - t->first_u[r]);
}

// CG start (x0 = 0): r = f, both direction buffers 0, r in the contraction-1
// operand layout (its padding is cleared beforehand), head partials
// (f.f, 0, 0); scalars for the iteration kernels.  FP64 path: 64 entries per
// block; BF16 forms: 128 (two per lane, split into BF16 terms in fragment
// order), matching the blocks of the update.
__device__ __forceinline__ void init_scalars(CgScalars* sc, double tol, int maxiter, double shift) {
    sc->done = 0;
    sc->bad = 0;
    sc->iters = 0;
    sc->it = 0;
    sc->tol = tol;
    sc->maxiter = maxiter;
    sc->shift = shift;
    sc->rr_prev = 0.0;
}

__global__ __launch_bounds__(64) void k_init3(Dims d, const double* __restrict__ f,
                                              double* __restrict__ x, double* __restrict__ r,
                                              double* __restrict__ p, double* __restrict__ p2,
                                              double* __restrict__ Rop, double* __restrict__ aux0,
                                              int nbv, double tol, int maxiter, double shift,
                                              CgScalars* sc) {
    const int total = d.Ma * d.Na;
    const int e = blockIdx.x * 64 + threadIdx.x;
    double q = 0.0;
    if (e < total) {
        const double fe = f[e];
        const int j = e / d.Na, i = e - j * d.Na;
        x[e] = 0.0;
        r[e] = fe;
        p[e] = 0.0;
        p2[e] = 0.0;
        Rop[(size_t)i * d.Ma + j] = fe;
        q = fe * fe;
    }
    q = wave_sum(q);
    if (threadIdx.x == 0) {
        aux0[blockIdx.x] = q;
        aux0[nbv + blockIdx.x] = 0.0;
        aux0[2 * (size_t)nbv + blockIdx.x] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) init_scalars(sc, tol, maxiter, shift);
}

__global__ __launch_bounds__(64) void k_init4(Dims d, const double* __restrict__ f,
                                              double* __restrict__ x, double* __restrict__ r,
                                              double* __restrict__ p, double* __restrict__ p2,
                                              uint16_t* __restrict__ Rop,
                                              double* __restrict__ aux0, int nbv, double tol,
                                              int maxiter, double shift, CgScalars* sc) {
    const int total = d.Ma * d.Na;
    const int e = blockIdx.x * 128 + 2 * threadIdx.x;
    double q = 0.0;
    if (e < total) {
        const double2 fe = *(const double2*)(f + e);
        const int j = e / d.Na, i = e - j * d.Na;
        const double2 z = make_double2(0.0, 0.0);
        *(double2*)(x + e) = z;
        *(double2*)(r + e) = fe;
        *(double2*)(p + e) = z;
        *(double2*)(p2 + e) = z;
        uint32_t hi, lo;
        split_pk((float)fe.x, (float)fe.y, hi, lo);
        const size_t o = pfrag_off(j, i, d.Kq / 128);
        *(uint32_t*)(Rop + o) = hi;
        *(uint32_t*)(Rop + (size_t)d.Ma * d.Kq + o) = lo;
        q = fe.x * fe.x + fe.y * fe.y;
    }
    q = wave_sum(q);
    if (threadIdx.x == 0) {
        aux0[blockIdx.x] = q;
        aux0[nbv + blockIdx.x] = 0.0;
        aux0[2 * (size_t)nbv + blockIdx.x] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) init_scalars(sc, tol, maxiter, shift);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int nb_of(long n, int b) { return (int)((n + b - 1) / b); }

long qgt_padded_samples(long n) { return (n + 511) / 512 * 512; }

size_t qgt_th_bytes(const Dims& d, int prec, long Nsp) {
    return (size_t)d.Ma * Nsp * (prec == 0 ? 8 : 4);
}

void launch_qgt_prepare(hipStream_t st, const Dims& d, int prec, const int8_t* s,
                        const void* tact, long n, const QgtBatch& q) {
    if (prec == 0) {
        const dim3 gs((unsigned)(q.Nsp / 64), (unsigned)nb_of(d.Kq, 64));
        k_prep_spins<<<gs, 256, 0, st>>>(s, d.N, n, d.Kb, d.Kq, q.Nsp, (int8_t*)q.Sp, q.St);
    } else {
        const dim3 gs((unsigned)(q.Nsp / 64), (unsigned)(d.Kq / 128));
        k_prep_spins4<<<gs, 256, 0, st>>>(s, d.N, n, d.Kb, d.Kq, q.Nsp, (uint8_t*)q.Sp,
                                          (uint8_t*)q.St);
    }
    const dim3 gt((unsigned)(q.Nsp / 64), (unsigned)nb_of(d.Ma, 64));
    if (prec == 0) {
        k_prep_t<double><<<gt, 256, 0, st>>>((const double*)tact, n, d.Mw, d.Ma, q.Nsp, q.Th);
    } else {
        k_prep_t<float><<<gt, 256, 0, st>>>((const float*)tact, n, d.Mw, d.Ma, q.Nsp, q.Th);
        const dim3 gf((unsigned)(q.Nsp / 64), (unsigned)(d.Ma / 16));
        k_prep_tf<<<gf, 256, 0, st>>>((const float*)tact, n, d.Mw, q.Tf);
    }
}

size_t qgt_spin_bytes(const Dims& d, int prec, long Nsp) {
    // Sp and St: one byte per spin (FP64 path) or one FP4 code (BF16 forms)
    return (size_t)Nsp * d.Kq / (prec == 0 ? 1 : 2);
}

int qgt_nbw(long n, int prec) {
    return nb_of(n, prec == 0 ? 16 * W5_RT : W7_ROWS);
}
long qgt_act_rows(long n) { return (n + W_ROWS_MAX - 1) / W_ROWS_MAX * W_ROWS_MAX; }
int qgt_nbu(const Dims& d) { return nb_of((long)d.Ma * d.Na, 256); }
int qgt_nbr(const Dims& d) { return nb_of((long)d.Ma * d.Na, 64); }
int qgt_nbv(const Dims& d, int prec) { return nb_of((long)d.Ma * d.Na, prec == 0 ? 64 : 128); }
size_t qgt_pop_bytes(const Dims& d, int prec) {
    return prec == 0 ? (size_t)d.Kq * d.Ma * 8 : (size_t)2 * d.Ma * d.Kq * 2;
}

void launch_qgt_w(hipStream_t st, const Dims& d, int prec, const QgtBatch& q, const void* tact,
                  long n, const void* Rop, double* w, const double* aux, CgScalars* sc) {
    int waves, per;
    wave_split(d.Ma / 16, prec == 0 ? 8 : 15, waves, per);
    const int nb = qgt_nbw(n, prec), nbv = qgt_nbv(d, prec);
    if (prec == 0) {
        k_w5<<<nb, 64 * waves, (size_t)16 * W5_RT * (d.Kb + 8), st>>>(d, (const int8_t*)q.Sp,
                                                                   (const double*)tact, n,
                                        (const double*)Rop, w, q.wpart, aux, nbv, sc);
    } else {  // one more wave for the CG head
        k_w7<<<nb, 64 * (waves + 1), 0, st>>>(d, (const uint8_t*)q.Sp, q.Tf, n,
                                              (const uint16_t*)Rop, w, q.wpart, aux, nbv, sc);
    }
}

int qgt_ksplit(const QgtBatch& q) { return q.ks; }

// FP64 contraction 2: site-tile passes of at most 32 tiles, tiles per pass,
// tiles per active wave, active waves and the block size
struct O9Shape {
    int passes, tpp, pt, nwa, nth;
};
static O9Shape o9_shape(const Dims& d) {
    const int ni = d.Na / 16;
    O9Shape s;
    s.passes = (ni + 31) / 32;
    s.tpp = (ni + s.passes - 1) / s.passes;
    s.pt = s.tpp > 16 ? 2 : 1;
    s.nwa = (s.tpp + s.pt - 1) / s.pt;
    s.nth = s.nwa > 8 ? 1024 : 512;
    return s;
}
void qgt_split(QgtBatch& q, const Dims& d, int prec, long n, int ncu) {
    if (prec != 0) {
        q.kc = O16_KC;
        q.ks = (int)(q.Nsp / q.kc);
        return;
    }
    // ranges per hidden tile: two 512-thread blocks or one 1024-thread block
    // per CU in all, each range at least one 16-sample unit
    const O9Shape sh = o9_shape(d);
    const long U = (n + 15) / 16, nj = d.Ma / 16;
    long ks = (sh.nth == 512 ? 2L : 1L) * (ncu > 0 ? ncu : 1) / (nj * sh.passes);
    ks = ks < 1 ? 1 : (ks > U ? U : ks);
    q.kc = 0;
    q.ks = (int)ks;
}

void launch_qgt_outer(hipStream_t st, const Dims& d, int prec, const QgtBatch& q, long n,
                      const double* v, int v_mode, void* part, double* papart,
                      const CgScalars* sc) {
    const int ks = qgt_ksplit(q), nj = d.Ma / 16, nbw = qgt_nbw(n, prec);
    if (prec == 0) {
        const O9Shape s = o9_shape(d);
        const int nb = s.passes * nj * ks;  // one block per work item, all in one round
#define O9_LAUNCH(PT, NTH)                                                                      \
    k_outer9<PT, NTH><<<nb, NTH, 0, st>>>(d, q.St, (const double*)q.Th, q.Nsp, n, v, v_mode,    \
                                          q.wpart, nbw, (double*)part, ks, s.tpp, s.nwa, papart, \
                                          sc)
        if (s.nth == 512)
            O9_LAUNCH(1, 512);
        else if (s.pt == 1)
            O9_LAUNCH(1, 1024);
        else
            O9_LAUNCH(2, 1024);
#undef O9_LAUNCH
    } else {
        const int nb = NXCD * nj * ((ks + NXCD - 1) / NXCD);
        k_outer8<<<nb, O8_THREADS, 0, st>>>(d, (const uint8_t*)q.St, (const float*)q.Th, q.Nsp, n,
                                            v, v_mode, q.wpart, nbw, (float*)part, ks, papart, sc);
    }
}

void launch_qgt_reduce(hipStream_t st, const Dims& d, int prec, const void* part, int ksplit,
                       const double* p, double shift, double* out, double* pap,
                       const CgScalars* sc, int cg) {
    const int nb = qgt_nbr(d);
    if (prec == 0)
        k_reduce3<double><<<nb, 256, 0, st>>>(d, (const double*)part, ksplit, p, shift, out, pap,
                                              sc, cg);
    else
        k_reduce3<float><<<nb, 256, 0, st>>>(d, (const float*)part, ksplit, p, shift, out, pap,
                                             sc, cg);
}

void launch_qgt_init(hipStream_t st, const Dims& d, int prec, const double* f, double* x,
                     double* r, double* p, double* p2, void* Rop, double* aux0, double* w, long n,
                     double tol, int maxiter, double shift, CgScalars* sc) {
    launch_zero(st, Rop, qgt_pop_bytes(d, prec));
    launch_zero(st, w, 8 * (size_t)n);
    const int nb = qgt_nbv(d, prec);
    if (prec == 0)
        k_init3<<<nb, 64, 0, st>>>(d, f, x, r, p, p2, (double*)Rop, aux0, nb, tol, maxiter, shift,
                                   sc);
    else
        k_init4<<<nb, 64, 0, st>>>(d, f, x, r, p, p2, (uint16_t*)Rop, aux0, nb, tol, maxiter,
                                   shift, sc);
}

int qgt_nbo(const Dims& d, const QgtBatch& q) { return qgt_ksplit(q); }

// slot slabs per wave the update loads up front for ks slots (4 waves)
static int update_sw(int ks) {
    const int per = (ks + 3) / 4;
    return per <= 4 ? 4 : per <= 8 ? 8 : per <= 12 ? 12 : 16;
}

void launch_qgt_update(hipStream_t st, const Dims& d, int prec, const QgtBatch& q,
                       const void* part, double* x, double* r, const double* p_old,
                       double* p_new, void* Rop, const double* papart, double* aux_next,
                       CgScalars* sc, int32_t* host_flag) {
    const int nb = qgt_nbv(d, prec), ks = qgt_ksplit(q), npa = qgt_nbo(d, q);
#define U4(SW)                                                                                 \
    k_update4<SW><<<nb, 256, 0, st>>>(d, (const double*)part, ks, x, r, p_old, p_new, Rop,   \
                                      papart, npa, aux_next, nb, sc, host_flag)
#define U5(SW)                                                                                 \
    k_update5<SW><<<nb, 256, 0, st>>>(d, (const float*)part, ks, x, r, p_old, p_new,         \
                                      (uint16_t*)Rop, papart, npa, aux_next, nb, sc, host_flag)
    const int sw = update_sw(ks);
    if (prec == 0) {
        if (sw == 4) U4(4);
        else if (sw == 8) U4(8);
        else if (sw == 12) U4(12);
        else U4(16);
    } else {
        if (sw == 4) U5(4);
        else if (sw == 8) U5(8);
        else if (sw == 12) U5(12);
        else U5(16);
    }
#undef U4
#undef U5
}

void cg_group_plan(CgGroupTable& t, CgGroupPlan& plan) {
    const int n = t.nrun;
    // one contraction-1 launch for every run, its blocks sized for the run with
    // the most contraction waves (plus the head wave); each run keeps its own
    int maxw = 1;
    for (int r = 0; r < n; ++r) {
        int waves, per;
        wave_split(t.run[r].d.Ma / 16, 15, waves, per);
        t.run[r].nwc = waves;
        maxw = std::max(maxw, waves);
    }
    plan.nw = 1;
    plan.w_base[0] = 0;
    plan.w_threads[0] = 64 * (maxw + 1);
    plan.u_sw = 4;
    int bw = 0, bo = 0, bu = 0;
    for (int r = 0; r < n; ++r) {
        const CgGroupRun& R = t.run[r];
        t.first_w[r] = bw;
        bw += qgt_nbw(R.n, 1);
        t.first_o[r] = bo;
        bo += NXCD * (R.d.Ma / 16) * ((R.ks + NXCD - 1) / NXCD);
        t.first_u[r] = bu;
        bu += qgt_nbv(R.d, 1);
        plan.u_sw = std::max(plan.u_sw, update_sw(R.ks));
    }
    for (int r = n; r < CG_GROUP_MAX; ++r) t.first_w[r] = t.first_o[r] = t.first_u[r] = INT_MAX;
    plan.w_blocks[0] = bw;
    plan.o_blocks = bo;
    plan.u_blocks = bu;
}

void launch_cg_group_iter(hipStream_t st, const CgGroupTable* t_dev, const CgGroupPlan& plan,
                          int par, int write_flag) {
    for (int g = 0; g < plan.nw; ++g)
        k_w7_group<<<plan.w_blocks[g], plan.w_threads[g], 0, st>>>(t_dev, plan.w_base[g], par);
    k_outer8_group<<<plan.o_blocks, O8_THREADS, 0, st>>>(t_dev);
    if (plan.u_sw == 4) k_update5_group<4><<<plan.u_blocks, 256, 0, st>>>(t_dev, par, write_flag);
    else if (plan.u_sw == 8) k_update5_group<8><<<plan.u_blocks, 256, 0, st>>>(t_dev, par, write_flag);
    else if (plan.u_sw == 12) k_update5_group<12><<<plan.u_blocks, 256, 0, st>>>(t_dev, par, write_flag);
    else k_update5_group<16><<<plan.u_blocks, 256, 0, st>>>(t_dev, par, write_flag);
}

}  // namespace nqs
