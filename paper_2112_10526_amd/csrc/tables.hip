// Parameter layout conversion, derived tables and chain starts.
#include "kernels.h"

namespace nqs {

void launch_zero(hipStream_t st, void* p, size_t bytes);

// packed boundary index -> augmented matrix position (see Dims)
__device__ __forceinline__ void packed_pos(const Dims& d, int idx, int& j, int& i) {
    if (d.vb) {
        if (idx < d.N) { j = d.M; i = idx; return; }
        idx -= d.N;
    }
    if (d.hb) {
        if (idx < d.M) { j = idx; i = d.N; return; }
        idx -= d.M;
    }
    j = idx / d.N;
    i = idx - j * d.N;
}

__global__ void k_unpack(Dims d, const double* __restrict__ p, double* __restrict__ Pm, int P) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P) return;
    int j, i;
    packed_pos(d, idx, j, i);
    Pm[(size_t)j * d.Na + i] = p[idx];
}

__global__ void k_pack(Dims d, const double* __restrict__ Pm, double* __restrict__ p, int P) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P) return;
    int j, i;
    packed_pos(d, idx, j, i);
    p[idx] = Pm[(size_t)j * d.Na + i];
}

// Zero every augmented entry that is not a parameter of this model.
__global__ void k_mask(Dims d, double* __restrict__ V) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d.Ma * d.Na) return;
    const int j = e / d.Na, i = e - j * d.Na;
    const bool keep = (j < d.M && i < d.N) || (d.hb && j < d.M && i == d.N) ||
                      (d.vb && j == d.M && i < d.N);
    if (!keep) V[e] = 0.0;
}

// T = tanh(2 W) in two layouts, and the theta-GEMM operand W~^T (rows i <= N,
// row N holding b), in the compute precision.
template <typename R>
__global__ void k_tables(Dims d, const double* __restrict__ Pm, R* __restrict__ Tt,
                         R* __restrict__ Tj, R* __restrict__ Wa) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;  // over Na * Mw
    if (e >= d.Na * d.Mw) return;
    const int i = e / d.Mw, j = e - i * d.Mw;
    const double w = (i <= d.N && j < d.M) ? Pm[(size_t)j * d.Na + i] : 0.0;
    Wa[e] = (R)w;
    if (i < d.N) {
        const double t = (j < d.M) ? tanh(2.0 * w) : 0.0;
        Tt[(size_t)i * d.Mw + j] = (R)t;
        Tj[(size_t)j * d.Nw + i] = (R)t;
    }
}

// BF16 two-term split of W~ stored hidden-major [Mw][Kb] (the K index is
// contiguous so one lane loads its eight K values with one 16-byte load).
__global__ void k_tables_bf16(Dims d, const double* __restrict__ Pm, uint16_t* __restrict__ Whi,
                              uint16_t* __restrict__ Wlo) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;  // over Mw * Kb
    if (e >= d.Kb * d.Mw) return;
    const int j = e / d.Kb, i = e - j * d.Kb;
    const float w = (i <= d.N && j < d.M) ? (float)Pm[(size_t)j * d.Na + i] : 0.0f;
    const uint16_t hi = f32_to_bf16_bits(w);
    Whi[e] = hi;
    Wlo[e] = f32_to_bf16_bits(w - bf16_bits_to_f32(hi));
}

// Site factors of the single-flip amplitude ratio:
//   psi(s with s_i flipped) / psi(s) = K_i(s_i) prod_j (1 - s_i tanh(theta_j) tanh(2 W_ji))
//   K_i(s) = exp(-2 a_i s) prod_j cosh(2 W_ji).
// FP64 tables hold K, FP32 tables hold ln K.  One wave per site.
template <typename R>
__global__ void k_site_consts(Dims d, const double* __restrict__ Pm, R* __restrict__ Ks) {
    const int site = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (site >= d.N) return;
    double acc = 0.0;
    for (int j = lane; j < d.M; j += 64) acc += log(cosh(2.0 * Pm[(size_t)j * d.Na + site]));
    acc = wave_sum(acc);
    if (lane == 0) {
        const double a = d.vb ? Pm[(size_t)d.M * d.Na + site] : 0.0;
        const double lp = acc - 2.0 * a, lm = acc + 2.0 * a;
        if (sizeof(R) == 8) {
            Ks[2 * site] = (R)exp(lp);
            Ks[2 * site + 1] = (R)exp(lm);
        } else {
            Ks[2 * site] = (R)lp;
            Ks[2 * site + 1] = (R)lm;
        }
    }
}

// Chain starts from the tag-1 Philox stream (one thread per chain).
// Random start: spin i is bit (i % 32) of word (i / 32) % 4 of the draw with
// counter (i / 128, 0, chain, 1); s = 1 - 2 bit.
// Zero-magnetisation start: N/2 up then N/2 down, Fisher-Yates shuffled; swap
// k exchanges position N-1-k with position floor(x0 * (N-k) / 2^32) of the
// draw with counter (k, 0, chain, 1).
__global__ void k_init_chains(int N, int C, uint64_t seed, int chain_offset, int sz0,
                              int8_t* __restrict__ s) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    int8_t* row = s + (size_t)c * N;
    const uint32_t g = (uint32_t)(chain_offset + c);
    if (!sz0) {
        for (int b = 0; b < N; b += 128) {
            const uint4 x = philox10(make_uint4((uint32_t)(b / 128), 0u, g, TAG_START), seed);
            const uint32_t w[4] = {x.x, x.y, x.z, x.w};
            for (int i = b; i < N && i < b + 128; ++i) {
                const uint32_t bit = (w[(i >> 5) & 3] >> (i & 31)) & 1u;
                row[i] = (int8_t)(1 - 2 * (int)bit);
            }
        }
    } else {
        for (int i = 0; i < N; ++i) row[i] = (int8_t)(i < N / 2 ? 1 : -1);
        for (int k = 0; k + 1 < N; ++k) {
            const int i = N - 1 - k;
            const uint4 x = philox10(make_uint4((uint32_t)k, 0u, g, TAG_START), seed);
            const int j = mulshift(x.x, i + 1);
            const int8_t t = row[i];
            row[i] = row[j];
            row[j] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int blocks(long n, int b) { return (int)((n + b - 1) / b); }

void launch_unpack(hipStream_t st, const Dims& d, const double* p, double* Pm, int P) {
    launch_zero(st, Pm, sizeof(double) * (size_t)d.Ma * d.Na);
    k_unpack<<<blocks(P, 256), 256, 0, st>>>(d, p, Pm, P);
}
void launch_pack(hipStream_t st, const Dims& d, const double* Pm, double* p, int P) {
    k_pack<<<blocks(P, 256), 256, 0, st>>>(d, Pm, p, P);
}
void launch_mask(hipStream_t st, const Dims& d, double* V) {
    k_mask<<<blocks((long)d.Ma * d.Na, 256), 256, 0, st>>>(d, V);
}
void launch_tables(hipStream_t st, const Dims& d, int prec, const double* Pm, const Tables& t) {
    const long n = (long)d.Na * d.Mw;
    if (prec == 0) {
        k_tables<double><<<blocks(n, 256), 256, 0, st>>>(d, Pm, (double*)t.Tt, (double*)t.Tj,
                                                         (double*)t.Wa);
        k_site_consts<double><<<blocks(d.N, 4), 256, 0, st>>>(d, Pm, (double*)t.Ks);
    } else {
        k_tables<float><<<blocks(n, 256), 256, 0, st>>>(d, Pm, (float*)t.Tt, (float*)t.Tj,
                                                        (float*)t.Wa);
        k_site_consts<float><<<blocks(d.N, 4), 256, 0, st>>>(d, Pm, (float*)t.Ks);
    }
    if (prec == 2) {
        const long nb = (long)d.Kb * d.Mw;
        k_tables_bf16<<<blocks(nb, 256), 256, 0, st>>>(d, Pm, t.Whi, t.Wlo);
    }
}
void launch_init_chains(hipStream_t st, int N, int C, uint64_t seed, int sz0, int8_t* s) {
    k_init_chains<<<blocks(C, 64), 64, 0, st>>>(N, C, seed, 0, sz0, s);
}

__global__ void k_zero(uint32_t* __restrict__ p, size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}
// Clear device memory with a kernel (safe inside captured graphs); bytes must
// be a multiple of 4.
void launch_zero(hipStream_t st, void* p, size_t bytes) {
    const size_t n = bytes / 4;
    if (!n) return;
    int nb = (int)((n + 255) / 256);
    if (nb > 4096) nb = 4096;
    k_zero<<<nb, 256, 0, st>>>((uint32_t*)p, n);
}

}  // namespace nqs
