// Dense-Jacobian form of the QGT (paper, QGTJacobianDense and its appendix):
// the Jacobian O[k][p] = d ln psi(s_k) / d p_p is materialised in the packed
// parameter order, centred and scaled (dJ = (O - mean O) / sqrt(N_s)), the
// Gram matrix G = dJ^T dJ is formed on MFMA, and CG runs on G v + eps v.
#include "kernels.h"

namespace nqs {

// O[k][p] for the packed layout [a | b | W]; row stride ld, zero padding to ld.
template <typename R>
__global__ __launch_bounds__(256) void k_jacobian(Dims d, const int8_t* __restrict__ s,
                                                  const R* __restrict__ tact, long n, int P,
                                                  long ld, R* __restrict__ O) {
    const long k = blockIdx.x;
    if (k >= n) return;
    const int8_t* sk = s + k * d.N;
    const R* tk = tact + k * d.Mw;
    R* row = O + k * ld;
    for (long p = threadIdx.x; p < ld; p += 256) {
        R v = (R)0;
        if (p < P) {
            long idx = p;
            if (d.vb) {
                if (idx < d.N) { row[p] = (R)sk[idx]; continue; }
                idx -= d.N;
            }
            if (d.hb) {
                if (idx < d.M) { row[p] = tk[idx]; continue; }
                idx -= d.M;
            }
            const long j = idx / d.N, i = idx - j * d.N;
            v = tk[j] * (R)sk[i];
        }
        row[p] = v;
    }
}

// colsum[p] = sum_k O[k][p] (fixed order down each column)
template <typename R>
__global__ void k_colsum(const R* __restrict__ O, long n, long ld, int P, double* __restrict__ cs) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double acc = 0.0;
    for (long k = 0; k < n; ++k) acc += (double)O[k * ld + p];
    cs[p] = acc;
}

// O <- (O - colsum / n) / sqrt(n)
template <typename R>
__global__ void k_center_scale(R* __restrict__ O, long n, long ld, int P,
                               const double* __restrict__ cs) {
    const long k = blockIdx.y;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || k >= n) return;
    const double inv = 1.0 / (double)n;
    const double rs = 1.0 / sqrt((double)n);
    R* e = O + k * ld + p;
    *e = (R)(((double)*e - cs[p] * inv) * rs);
}

// G[p][q] = sum_k A[k][p] A[k][q] for the upper block triangle, mirrored.
// Block = 4 waves = a 128 x 128 tile of G; each wave a 64 x 64 quarter as
// 4 x 4 MFMA tiles of 16 x 16 sharing its operand fragments.
template <typename R>
__global__ __launch_bounds__(256) void k_gram(const R* __restrict__ A, long n, long ld, int P,
                                              R* __restrict__ G, const int* __restrict__ tiles) {
    const int tp = tiles[2 * blockIdx.x], tq = tiles[2 * blockIdx.x + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int p0 = tp * 128 + (wave >> 1) * 64;
    const int q0 = tq * 128 + (wave & 1) * 64;
    typedef typename std::conditional<sizeof(R) == 8, v4d, v4f>::type acc_t;
    acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    for (long k0 = 0; k0 < n; k0 += 4) {
        const long k = k0 + lk;
        R fa[4], fb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const long p = p0 + a * 16 + lr, q = q0 + a * 16 + lr;
            fa[a] = (k < n && p < ld) ? A[k * ld + p] : (R)0;
            fb[a] = (k < n && q < ld) ? A[k * ld + q] : (R)0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if constexpr (sizeof(R) == 8)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
                else
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[b], acc[a][b], 0, 0, 0);
            }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long p = p0 + a * 16 + acc_row<R>(lk, i), q = q0 + b * 16 + lr;
                if (p < P && q < P) {
                    G[p * ld + q] = acc[a][b][i];
                    if (tp != tq) G[q * ld + p] = acc[a][b][i];
                }
            }
}

template <int NT>
__device__ __forceinline__ double bsum(double v, double* sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// out = G v + shift v (FP64 accumulation), one wave per row; last block forms
// alpha = rr / (v . out).
template <typename R>
__global__ __launch_bounds__(256) void k_dense_matvec(const R* __restrict__ G, int P, long ld,
                                                      const double* __restrict__ v, double shift,
                                                      double* __restrict__ out,
                                                      double* __restrict__ dpart, CgScalars* sc) {
    if (sc->done) return;
    __shared__ double sh[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long p = (long)blockIdx.x * 4 + wave;
    double dot = 0.0;
    if (p < P) {
        const R* row = G + p * ld;
        double acc = 0.0;
        for (long q = lane; q < P; q += 64) acc += (double)row[q] * v[q];
        acc = wave_sum(acc) + shift * v[p];
        if (lane == 0) out[p] = acc;
        dot = lane == 0 ? acc * v[p] : 0.0;
    }
    dot = bsum<256>(dot, sh);
    if (threadIdx.x == 0) dpart[blockIdx.x] = dot;
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = (atomicAdd(&sc->counter[3], 1u) == gridDim.x - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    double a = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += 256) a += *(const volatile double*)&dpart[b];
    const double pap = bsum<256>(a, sh);
    if (threadIdx.x == 0) {
        sc->pAp = pap;
        sc->alpha = sc->rr / pap;
        if (!(pap > 0.0) || !isfinite(sc->alpha)) { sc->bad = 1; sc->done = 1; }
        sc->counter[3] = 0;
    }
}

// ---------------------------------------------------------------------------
void launch_jacobian(hipStream_t st, const Dims& d, int prec, const int8_t* s, const void* tact,
                     long n, void* O, int P, long ld) {
    if (n <= 0) return;
    if (prec == 0)
        k_jacobian<double><<<(unsigned)n, 256, 0, st>>>(d, s, (const double*)tact, n, P, ld,
                                                        (double*)O);
    else
        k_jacobian<float><<<(unsigned)n, 256, 0, st>>>(d, s, (const float*)tact, n, P, ld,
                                                       (float*)O);
}

void launch_center_cols(hipStream_t st, int prec, void* O, long n, long ld, int P, double* cs) {
    const int nb = (P + 255) / 256;
    const dim3 g2(nb, (unsigned)n);
    if (prec == 0) {
        k_colsum<double><<<nb, 256, 0, st>>>((const double*)O, n, ld, P, cs);
        k_center_scale<double><<<g2, 256, 0, st>>>((double*)O, n, ld, P, cs);
    } else {
        k_colsum<float><<<nb, 256, 0, st>>>((const float*)O, n, ld, P, cs);
        k_center_scale<float><<<g2, 256, 0, st>>>((float*)O, n, ld, P, cs);
    }
}

int gram_tiles(int P) {
    const int nt = (P + 127) / 128;
    return nt * (nt + 1) / 2;
}
void fill_gram_tiles(int P, int* host_tiles) {
    const int nt = (P + 127) / 128;
    int e = 0;
    for (int a = 0; a < nt; ++a)
        for (int b = a; b < nt; ++b) {
            host_tiles[2 * e] = a;
            host_tiles[2 * e + 1] = b;
            ++e;
        }
}
void launch_gram(hipStream_t st, int prec, const void* A, long n, long ld, int P, void* G,
                 const int* tiles, int ntiles) {
    if (prec == 0)
        k_gram<double><<<ntiles, 256, 0, st>>>((const double*)A, n, ld, P, (double*)G, tiles);
    else
        k_gram<float><<<ntiles, 256, 0, st>>>((const float*)A, n, ld, P, (float*)G, tiles);
}
void launch_dense_matvec(hipStream_t st, int prec, const void* G, int P, long ld, const double* v,
                         double shift, double* out, double* dpart, CgScalars* sc) {
    const int nb = (P + 3) / 4;
    if (prec == 0)
        k_dense_matvec<double><<<nb, 256, 0, st>>>((const double*)G, P, ld, v, shift, out, dpart, sc);
    else
        k_dense_matvec<float><<<nb, 256, 0, st>>>((const float*)G, P, ld, v, shift, out, dpart, sc);
}

}  // namespace nqs
