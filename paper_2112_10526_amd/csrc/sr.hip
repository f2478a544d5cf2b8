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

// Stage rows [k0, k0 + rows) of the augmented spins (s, 1, 0 ...) into
// LDS [rows][Na]; rows at or beyond kend are zero.  Source rows are
// contiguous, so the copy is a flat byte stream read 16 bytes per lane.
__device__ __forceinline__ void stage_spins(int8_t* __restrict__ Ss, const int8_t* __restrict__ s,
                                            int N, int Na, long k0, int rows, long kend) {
    const int tid = threadIdx.x;
    const long nrow = max(0L, min((long)rows, kend - k0));
    const long total = nrow * N;
    const int8_t* src = s + k0 * N;
    for (long base = 0; base < total; base += 256 * 16) {
        int8_t b[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const long e = base + u * 256 + tid;
            b[u] = e < total ? src[e] : (int8_t)0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const long e = base + u * 256 + tid;
            if (e < total) {
                const int rl = (int)(e / N), i = (int)(e - (long)rl * N);
                Ss[rl * Na + i] = b[u];
            }
        }
    }
    // augmented columns and rows past the end
    for (int e = tid; e < rows * (Na - N); e += 256) {
        const int rl = e / (Na - N), i = N + (e - rl * (Na - N));
        Ss[rl * Na + i] = (rl < nrow && i == N) ? (int8_t)1 : (int8_t)0;
    }
    for (long e = nrow * Na + tid; e < (long)rows * Na; e += 256) Ss[e] = 0;
}

// ---------------------------------------------------------------------------
// contraction 2: part[kc][j][i] = sum_{k in chunk kc} t~_kj z_k s~_ki
// z_k = (w_k - mean w) / n (v_mode 0, QGT product) or z_k = v_k (v_mode 1).
// grid = (ceil(Ma / (16 JG)), ksplit).  The block stages t~ z for its chunk
// of samples and JG hidden tiles, and the chunk's spins, in LDS; wave w owns
// hidden tile w % JG and every (4/JG)-th site tile starting at w / JG.
// ---------------------------------------------------------------------------
template <typename R, int JG>
__global__ __launch_bounds__(256) void k_outer(Dims d, const int8_t* __restrict__ s,
                                               const R* __restrict__ tact, long n,
                                               const double* __restrict__ v, int v_mode,
                                               R* __restrict__ part, int chunk,
                                               const CgScalars* __restrict__ sc) {
    if (v_mode == 0 && sc->done) return;
    extern __shared__ __align__(16) char lds_raw[];
    constexpr int JW = 16 * JG;  // hidden rows staged
    constexpr int IG = 4 / JG;   // site-tile groups
    const int Na = d.Na;
    const int KC = (chunk + 3) / 4 * 4;
    R* Ts = (R*)lds_raw;                     // [KC][JW]
    int8_t* Ss = (int8_t*)(Ts + KC * JW);    // [KC][Na]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    double shift = 0.0, scale = 1.0;
    if (v_mode == 0) {
        shift = sc->wmean;
        scale = 1.0 / (double)n;
    }
    const long kbeg = (long)blockIdx.y * chunk;
    const int kn = (int)max(0L, min((long)chunk, n - kbeg));
    const int j0 = blockIdx.x * JW;
    R* zs = (R*)(Ss + KC * Na + 16 - ((KC * Na) & 15));  // [KC] scaled z, 16-byte aligned
    for (int kl = tid; kl < KC; kl += 256)
        zs[kl] = kl < kn ? (R)((v[kbeg + kl] - shift) * scale) : (R)0;
    stage_spins(Ss, s, d.N, Na, kbeg, KC, kbeg + kn);
    __syncthreads();
    for (int base = 0; base < KC * JW; base += 256 * 8) {
        R t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + u * 256 + tid;
            const int kl = e / JW, j = j0 + (e - kl * JW);
            t[u] = (kl < kn && j < d.Ma) ? tact[(kbeg + kl) * d.Mw + j] : (R)0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + u * 256 + tid;
            if (e < KC * JW) Ts[e] = t[u] * zs[e / JW];
        }
    }
    __syncthreads();
    const int jt = blockIdx.x * JG + wave % JG;
    if (jt * 16 >= d.Ma) return;
    const int nct = Na / 16;
    typedef typename std::conditional<sizeof(R) == 8, v4d, v4f>::type acc_t;
    R* out = part + (size_t)blockIdx.y * d.Ma * Na;
    const R* Tw = Ts + (wave % JG) * 16 + lr;
    for (int ct0 = wave / JG; ct0 < nct; ct0 += IG * 8) {
        acc_t acc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = acc_t{0, 0, 0, 0};
        for (int k0 = 0; k0 < KC; k0 += 4) {
            const R a = Tw[(k0 + lk) * JW];
            const int8_t* Sk = Ss + (k0 + lk) * Na + lr;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int ct = ct0 + c * IG;
                if (ct < nct) {
                    const R b = (R)Sk[ct * 16];
                    if constexpr (sizeof(R) == 8)
                        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
                    else
                        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int ct = ct0 + c * IG;
            if (ct < nct) {
                const int i = ct * 16 + lr;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int jj = jt * 16 + acc_row<R>(lk, q);
                    out[(size_t)jj * Na + i] = acc[c][q];
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
            int kc = 0;
            for (; kc + 8 <= ksplit; kc += 8) {
                R x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = part[(size_t)(kc + u) * total + e];
#pragma unroll
                for (int u = 0; u < 8; ++u) val += (double)x[u];
            }
            for (; kc < ksplit; ++kc) val += (double)part[(size_t)kc * total + e];
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

// Dense-form CG, one iteration in three kernels (product, update, direction);
// each sums the block partials of the kernel before it in a fixed order (the
// same in every block), so no kernel needs a cross-block step:
//   update:    p.Ap from the product's partials, alpha = r.r / p.Ap,
//              x += alpha p, r -= alpha Ap, block partials of the new r.r;
//   direction: r.r from the update's partials, beta = r.r / r.r_prev,
//              p = r + beta p; block 0 advances the iteration and the stop flag
//              (also stored to a pinned host word when asked: the last
//              iteration of a batch, so a batch can be replayed from a graph).
// The diagonal shift is taken from the scalars (set by k_cg_init).
// Every scalar is written by a different kernel from the one that reads it.
__device__ __forceinline__ double sum_partials(const double* part, int np, double* sh) {
    double a = 0.0;
    for (int b = threadIdx.x; b < np; b += 256) a += part[b];
    return block_sum<256>(a, sh);
}
__global__ __launch_bounds__(256) void k_cg_update(int total, double* __restrict__ x,
                                                   double* __restrict__ r,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ Ap,
                                                   const double* __restrict__ pap_part, int npap,
                                                   double* __restrict__ rr_part, CgScalars* sc) {
    if (sc->done) return;
    __shared__ double sh[4];
    const int e = blockIdx.x * 256 + threadIdx.x;
    const double rr = sc->rr;
    const double pAp = sum_partials(pap_part, npap, sh);
    const double alpha = rr / pAp;
    if (!(pAp > 0.0) || !isfinite(alpha)) {  // the same decision in every block
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->bad = 1;
            sc->done = 1;
        }
        return;
    }
    double rn = 0.0;
    if (e < total) {
        x[e] += alpha * p[e];
        const double re = r[e] - alpha * Ap[e];
        r[e] = re;
        rn = re * re;
    }
    rn = block_sum<256>(rn, sh);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = rn;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->alpha = alpha;
        sc->pAp = pAp;
        sc->rr_prev = rr;
    }
}

__global__ __launch_bounds__(256) void k_cg_p(int total, const double* __restrict__ r,
                                              double* __restrict__ p,
                                              const double* __restrict__ rr_part, int nrr,
                                              CgScalars* sc, volatile int32_t* host_flag) {
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (sc->done) {
        if (host_flag && lead) *host_flag = 1;
        return;
    }
    __shared__ double sh[4];
    const double rr = sum_partials(rr_part, nrr, sh);
    const double beta = rr / sc->rr_prev;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < total) p[e] = r[e] + beta * p[e];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->beta = beta;
        sc->rr = rr;
        sc->iters += 1;
        if (!isfinite(rr)) {
            sc->bad = 1;
            sc->done = 1;
        }
        if (rr <= sc->tol2 || sc->iters >= sc->maxiter) sc->done = 1;
        if (host_flag) *host_flag = sc->done;
    }
}

// x = 0, r = p = f, rr = f.f, thresholds.
__global__ __launch_bounds__(256) void k_cg_init(int total, const double* __restrict__ f,
                                                 double* __restrict__ x, double* __restrict__ r,
                                                 double* __restrict__ p, double* __restrict__ dpart,
                                                 CgScalars* sc, double tol, int maxiter,
                                                 double shift) {
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
            sc->beta = 0.0;
            sc->tol2 = tol * tol * s;
            sc->iters = 0;
            sc->maxiter = maxiter;
            sc->shift = shift;
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
template <typename K>
static void allow_lds(K kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bytes);
}
size_t outer_lds_bytes(const Dims& d, int prec, int chunk) {
    const int KC = (chunk + 3) / 4 * 4;
    const int JW = prec == 0 ? 32 : 64;
    const size_t es = prec == 0 ? 8 : 4;
    return (size_t)KC * JW * es + (size_t)KC * d.Na + 16 + (size_t)KC * es;
}
// Samples per chunk of contraction 2: up to 256, within the LDS limit.
int outer_chunk(const Dims& d, int prec, size_t lds_limit) {
    int c = 256;
    while (c > 16 && outer_lds_bytes(d, prec, c) > lds_limit) c -= 16;
    return c;
}
int outer_ksplit(long n, int chunk) {
    long ks = (n + chunk - 1) / chunk;
    return ks < 1 ? 1 : (int)ks;
}
void launch_outer(hipStream_t st, const Dims& d, int prec, const int8_t* s, const void* tact,
                  long n, const double* v, int v_mode, void* part, int chunk,
                  const CgScalars* sc) {
    const int ksplit = outer_ksplit(n, chunk);
    const size_t lds = outer_lds_bytes(d, prec, chunk);
    if (prec == 0) {
        const dim3 grid(nblk(d.Ma, 32), ksplit);
        allow_lds(k_outer<double, 2>, lds);
        k_outer<double, 2><<<grid, 256, lds, st>>>(d, s, (const double*)tact, n, v, v_mode,
                                                   (double*)part, chunk, sc);
    } else {
        const dim3 grid(nblk(d.Ma, 64), ksplit);
        allow_lds(k_outer<float, 4>, lds);
        k_outer<float, 4><<<grid, 256, lds, st>>>(d, s, (const float*)tact, n, v, v_mode,
                                                  (float*)part, chunk, sc);
    }
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
                    double* dpart, CgScalars* sc, double tol, int maxiter, double shift) {
    k_cg_init<<<nblk(total, 256), 256, 0, st>>>(total, f, x, r, p, dpart, sc, tol, maxiter, shift);
}
void launch_cg_update(hipStream_t st, int total, double* x, double* r, double* p,
                      const double* Ap, double* dpart, int npap, CgScalars* sc,
                      int32_t* host_flag) {
    const int nb = nblk(total, 256);
    double* rr_part = dpart + npap;  // after the product's partials
    k_cg_update<<<nb, 256, 0, st>>>(total, x, r, p, Ap, dpart, npap, rr_part, sc);
    k_cg_p<<<nb, 256, 0, st>>>(total, r, p, rr_part, nb, sc, host_flag);
}
void launch_axpy_update(hipStream_t st, int total, double* x, const double* delta, double lr,
                        CgScalars* sc) {
    k_axpy_update<<<nblk(total, 256), 256, 0, st>>>(total, x, delta, lr, sc);
}

}  // namespace nqs
