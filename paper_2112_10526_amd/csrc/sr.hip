// Energy statistics, force, on-the-fly QGT products and conjugate gradients.
//
// With the augmented layout (see common.h) the log-derivatives of sample k
// form the outer product O_k = t~_k (x) s~_k, an [Ma][Na] matrix.  Hence
//   (J v)_k  = sum_j t~_kj sum_i s~_ki V[j][i]                 (contraction 1)
//   (J^T z)  = sum_k z_k t~_k (x) s~_k = T~^T diag(z) S~        (contraction 2)
// The on-the-fly QGT product of the paper's appendix,
//   w = J v / N_s,  dw = w - mean(w),  G v = J^T dw,
// and the force 2 Cov[O, E] = (2/N_s) J^T (E - mean E) are both contraction 2
// with a different z; contraction 1 gives w.  Both run on MFMA (FP64 16x16x4
// for the FP64 path, FP32 16x16x4 otherwise).  Contraction 2 is split over
// sample chunks; the chunk partials are summed in a fixed order, and every
// other reduction (means, dot products) is a fixed-order two-level sum, so
// results do not depend on timing or on what else runs on the device.
#include "kernels.h"

namespace nqs {

// ---------------------------------------------------------------------------
// block-level helpers
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[wave] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// true in exactly one block: the last to arrive; its earlier writes and all
// other blocks' writes before their arrival are visible to it afterwards.
__device__ __forceinline__ bool arrive_last(uint32_t* counter) {
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t v = atomicAdd(counter, 1u);
        last = (v == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (last) __threadfence();
    return last != 0;
}

__device__ __forceinline__ double vload(const double* p) { return *(const volatile double*)p; }

// Fixed-order sum of nb block partials by one 256-thread block.
__device__ __forceinline__ double final_sum(const double* dpart, int nb, double* sh) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) a += vload(&dpart[b]);
    return block_sum<256>(a, sh);
}

// ---------------------------------------------------------------------------
// statistics: mean, variance (1/n) and error of the mean; one block
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_stats(const double* __restrict__ E, long n,
                                                double* __restrict__ out) {
    __shared__ double sh[16];
    double a = 0.0;
    for (long k = threadIdx.x; k < n; k += 1024) a += E[k];
    const double mean = block_sum<1024>(a, sh) / (double)n;
    double b = 0.0;
    for (long k = threadIdx.x; k < n; k += 1024) {
        const double d = E[k] - mean;
        b += d * d;
    }
    const double var = block_sum<1024>(b, sh) / (double)n;
    if (threadIdx.x == 0) {
        out[0] = mean;
        out[1] = var;
        out[2] = sqrt(var / (double)n);
    }
}

// v_k = scale * (E_k - mean)
__global__ void k_center(const double* __restrict__ E, const double* __restrict__ stats,
                         double scale, long n, double* __restrict__ v) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) v[k] = scale * (E[k] - stats[0]);
}

// ---------------------------------------------------------------------------
// contraction 1: w_k = t~_k . (V s~_k), V = current CG direction [Ma][Na]
// One block = 4 waves = 64 samples; every wave: 16 samples x all Ma rows of V,
// 8 column tiles of 16 hidden units at a time.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R spin_aug(const int8_t* __restrict__ s, int N, long k, long n, int i) {
    if (k >= n || i > N) return (R)0;
    return i == N ? (R)1 : (R)s[k * N + i];
}

template <typename R>
__global__ __launch_bounds__(256) void k_qgt_w(Dims d, const int8_t* __restrict__ s,
                                               const R* __restrict__ tact, long n,
                                               const double* __restrict__ V,
                                               double* __restrict__ w, double* __restrict__ wpart,
                                               CgScalars* sc) {
    if (sc->done) return;
    __shared__ double sh[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long row0 = (long)blockIdx.x * 64 + wave * 16;
    typedef typename std::conditional<sizeof(R) == 8, v4d, v4f>::type acc_t;
    R wacc[4] = {0, 0, 0, 0};
    const int nct = d.Ma / 16;
    for (int ct0 = 0; ct0 < nct; ct0 += 8) {
        acc_t acc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = acc_t{0, 0, 0, 0};
        for (int k0 = 0; k0 < d.Na; k0 += 4) {
            const int i = k0 + lk;
            const R a = spin_aug<R>(s, d.N, row0 + lr, n, i);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if (ct0 + c < nct) {
                    const int j = (ct0 + c) * 16 + lr;
                    const R b = (R)V[(size_t)j * d.Na + i];
                    if constexpr (sizeof(R) == 8)
                        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
                    else
                        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (ct0 + c < nct) {
                const int j = (ct0 + c) * 16 + lr;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const long k = row0 + acc_row<R>(lk, q);
                    const R t = k < n ? tact[k * d.Mw + j] : (R)0;
                    wacc[q] += t * acc[c][q];
                }
            }
        }
    }
    double wsum = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double v = row16_sum((double)wacc[q]);
        const long k = row0 + acc_row<R>(lk, q);
        if (lr == 0 && k < n) w[k] = v;
        if (lr == 0 && k < n) wsum += v;
    }
    // block partial of sum_k w_k (lanes 0, 16, 32, 48 carry the row sums);
    // the last block turns the partials into mean(w)
    wsum = block_sum<256>(wsum, sh);
    if (threadIdx.x == 0) wpart[blockIdx.x] = wsum;
    if (arrive_last(&sc->counter[4])) {
        const double tot = final_sum(wpart, gridDim.x, sh);
        if (threadIdx.x == 0) {
            sc->wmean = tot / (double)n;
            sc->counter[4] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// contraction 2: part[kc][j][i] = sum_{k in chunk kc} t~_kj z_k s~_ki
// z_k = (w_k - mean w) / n (v_mode 0, QGT product) or z_k = v_k (v_mode 1).
// grid = (ceil(Ma / 64), ksplit); each wave owns one 16-row tile of hidden
// units and walks the Na site columns 8 tiles at a time.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_outer(Dims d, const int8_t* __restrict__ s,
                                               const R* __restrict__ tact, long n,
                                               const double* __restrict__ v, int v_mode,
                                               R* __restrict__ part, long chunk,
                                               const CgScalars* __restrict__ sc) {
    if (v_mode == 0 && sc->done) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int jt = blockIdx.x * 4 + wave;  // hidden-unit tile
    if (jt * 16 >= d.Ma) return;
    double shift = 0.0, scale = 1.0;
    if (v_mode == 0) {
        shift = sc->wmean;
        scale = 1.0 / (double)n;
    }
    const long kbeg = (long)blockIdx.y * chunk;
    const long kend = min(n, kbeg + chunk);
    const int j = jt * 16 + lr;
    typedef typename std::conditional<sizeof(R) == 8, v4d, v4f>::type acc_t;
    const int nct = d.Na / 16;
    R* out = part + (size_t)blockIdx.y * d.Ma * d.Na;
    for (int ct0 = 0; ct0 < nct; ct0 += 8) {
        acc_t acc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = acc_t{0, 0, 0, 0};
        for (long k0 = kbeg; k0 < kend; k0 += 4) {
            const long k = k0 + lk;
            R a = (R)0;
            if (k < kend) a = tact[k * d.Mw + j] * (R)((v[k] - shift) * scale);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if (ct0 + c < nct) {
                    const int i = (ct0 + c) * 16 + lr;
                    const R b = k < kend ? spin_aug<R>(s, d.N, k, n, i) : (R)0;
                    if constexpr (sizeof(R) == 8)
                        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
                    else
                        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (ct0 + c < nct) {
                const int i = (ct0 + c) * 16 + lr;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int jj = jt * 16 + acc_row<R>(lk, q);
                    out[(size_t)jj * d.Na + i] = acc[c][q];
                }
            }
        }
    }
}

// out[e] = sum_kc part[kc][e] + shift * p[e], masked to parameter entries.
// mode 0 (CG): also p . out -> alpha = rr / pAp in the last block.
template <typename R>
__global__ __launch_bounds__(256) void k_reduce_outer(Dims d, const R* __restrict__ part,
                                                      int ksplit, const double* __restrict__ p,
                                                      double shift, double* __restrict__ out,
                                                      double* __restrict__ dpart, CgScalars* sc,
                                                      int mode) {
    if (mode == 0 && sc->done) return;
    __shared__ double sh[4];
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int total = d.Ma * d.Na;
    double val = 0.0, dot = 0.0;
    if (e < total) {
        const int j = e / d.Na, i = e - j * d.Na;
        const bool keep = (j < d.M && i < d.N) || (d.hb && j < d.M && i == d.N) ||
                          (d.vb && j == d.M && i < d.N);
        if (keep) {
            for (int kc = 0; kc < ksplit; ++kc) val += (double)part[(size_t)kc * total + e];
            if (p) val += shift * p[e];
        }
        out[e] = val;
        if (mode == 0) dot = val * p[e];
    }
    if (mode != 0) return;
    dot = block_sum<256>(dot, sh);
    if (threadIdx.x == 0) dpart[blockIdx.x] = dot;
    if (arrive_last(&sc->counter[0])) {
        const double pap = final_sum(dpart, gridDim.x, sh);
        if (threadIdx.x == 0) {
            sc->pAp = pap;
            sc->alpha = sc->rr / pap;
            if (!(pap > 0.0) || !isfinite(sc->alpha)) { sc->bad = 1; sc->done = 1; }
            sc->counter[0] = 0;
        }
    }
}

// x += alpha p ; r -= alpha Ap ; rr' = r.r -> beta, convergence test.
__global__ __launch_bounds__(256) void k_cg_update(int total, double* __restrict__ x,
                                                   double* __restrict__ r,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ Ap,
                                                   double* __restrict__ dpart, CgScalars* sc) {
    if (sc->done) return;
    __shared__ double sh[4];
    const int e = blockIdx.x * 256 + threadIdx.x;
    const double alpha = sc->alpha;
    double rr = 0.0;
    if (e < total) {
        x[e] += alpha * p[e];
        const double re = r[e] - alpha * Ap[e];
        r[e] = re;
        rr = re * re;
    }
    rr = block_sum<256>(rr, sh);
    if (threadIdx.x == 0) dpart[blockIdx.x] = rr;
    if (arrive_last(&sc->counter[1])) {
        const double s = final_sum(dpart, gridDim.x, sh);
        if (threadIdx.x == 0) {
            sc->beta = s / sc->rr;
            sc->rr = s;
            sc->iters += 1;
            if (!isfinite(s)) { sc->bad = 1; sc->done = 1; }
            if (s <= sc->tol2 || sc->iters >= sc->maxiter) sc->done = 1;
            sc->counter[1] = 0;
        }
    }
}

// p = r + beta p
__global__ __launch_bounds__(256) void k_cg_p(int total, const double* __restrict__ r,
                                              double* __restrict__ p, const CgScalars* sc) {
    if (sc->done) return;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < total) p[e] = r[e] + sc->beta * p[e];
}

// x = 0, r = p = f, rr = f.f, thresholds.
__global__ __launch_bounds__(256) void k_cg_init(int total, const double* __restrict__ f,
                                                 double* __restrict__ x, double* __restrict__ r,
                                                 double* __restrict__ p, double* __restrict__ dpart,
                                                 CgScalars* sc, double tol, int maxiter) {
    __shared__ double sh[4];
    const int e = blockIdx.x * 256 + threadIdx.x;
    double ff = 0.0;
    if (e < total) {
        const double fe = f[e];
        x[e] = 0.0;
        r[e] = fe;
        p[e] = fe;
        ff = fe * fe;
    }
    ff = block_sum<256>(ff, sh);
    if (threadIdx.x == 0) dpart[blockIdx.x] = ff;
    if (arrive_last(&sc->counter[2])) {
        const double s = final_sum(dpart, gridDim.x, sh);
        if (threadIdx.x == 0) {
            sc->rr = s;
            sc->rr0 = s;
            sc->tol2 = tol * tol * s;
            sc->iters = 0;
            sc->maxiter = maxiter;
            sc->bad = isfinite(s) ? 0 : 1;
            sc->done = (s <= sc->tol2 || maxiter <= 0 || !isfinite(s)) ? 1 : 0;
            sc->counter[2] = 0;
        }
    }
}

// Pm -= lr * delta (delta is zero outside parameter entries); flags non-finite.
__global__ void k_axpy_update(int total, double* __restrict__ Pm, const double* __restrict__ delta,
                              double lr, CgScalars* sc) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const double v = Pm[e] - lr * delta[e];
    Pm[e] = v;
    if (!isfinite(v)) sc->bad = 2;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

void launch_stats(hipStream_t st, const double* E, long n, double* out3) {
    k_stats<<<1, 1024, 0, st>>>(E, n, out3);
}
void launch_center(hipStream_t st, const double* E, const double* stats, double scale, long n,
                   double* v) {
    k_center<<<nblk(n, 256), 256, 0, st>>>(E, stats, scale, n, v);
}
void launch_w(hipStream_t st, const Dims& d, int prec, const int8_t* s, const void* tact, long n,
              const double* V, double* w, double* wpart, CgScalars* sc) {
    const int nb = nblk(n, 64);
    if (prec == 0)
        k_qgt_w<double><<<nb, 256, 0, st>>>(d, s, (const double*)tact, n, V, w, wpart, sc);
    else
        k_qgt_w<float><<<nb, 256, 0, st>>>(d, s, (const float*)tact, n, V, w, wpart, sc);
}
int outer_ksplit(long n) {
    // about 256 samples per chunk, at most 64 chunks
    long ks = (n + 255) / 256;
    if (ks > 64) ks = 64;
    if (ks < 1) ks = 1;
    return (int)ks;
}
void launch_outer(hipStream_t st, const Dims& d, int prec, const int8_t* s, const void* tact,
                  long n, const double* v, int v_mode, void* part, int ksplit,
                  const CgScalars* sc) {
    long chunk = (n + ksplit - 1) / ksplit;
    chunk = (chunk + 3) / 4 * 4;
    const dim3 grid(nblk(d.Ma, 64), ksplit);
    if (prec == 0)
        k_outer<double><<<grid, 256, 0, st>>>(d, s, (const double*)tact, n, v, v_mode,
                                              (double*)part, chunk, sc);
    else
        k_outer<float><<<grid, 256, 0, st>>>(d, s, (const float*)tact, n, v, v_mode,
                                             (float*)part, chunk, sc);
}
void launch_reduce_outer(hipStream_t st, const Dims& d, int prec, const void* part, int ksplit,
                         const double* p, double shift, double* out, double* dpart,
                         CgScalars* sc, int mode) {
    const int nb = nblk((long)d.Ma * d.Na, 256);
    if (prec == 0)
        k_reduce_outer<double><<<nb, 256, 0, st>>>(d, (const double*)part, ksplit, p, shift, out,
                                                   dpart, sc, mode);
    else
        k_reduce_outer<float><<<nb, 256, 0, st>>>(d, (const float*)part, ksplit, p, shift, out,
                                                  dpart, sc, mode);
}
void launch_cg_init(hipStream_t st, int total, const double* f, double* x, double* r, double* p,
                    double* dpart, CgScalars* sc, double tol, int maxiter) {
    k_cg_init<<<nblk(total, 256), 256, 0, st>>>(total, f, x, r, p, dpart, sc, tol, maxiter);
}
void launch_cg_update(hipStream_t st, int total, double* x, double* r, double* p,
                      const double* Ap, double* dpart, CgScalars* sc) {
    k_cg_update<<<nblk(total, 256), 256, 0, st>>>(total, x, r, p, Ap, dpart, sc);
    k_cg_p<<<nblk(total, 256), 256, 0, st>>>(total, r, p, sc);
}
void launch_axpy_update(hipStream_t st, int total, double* x, const double* delta, double lr,
                        CgScalars* sc) {
    k_axpy_update<<<nblk(total, 256), 256, 0, st>>>(total, x, delta, lr, sc);
}

}  // namespace nqs
