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
//   Sp  int8 [Nsp][Kb]  augmented spins, sample-major   (contraction 1, A)
//   St  int8 [Kb][Nsp]  augmented spins, site-major     (contraction 2, B)
//   Th  [Ma][Nsp]       t~ hidden-major: FP64, or two BF16 planes hi/lo
// FP64 path: v_mfma_f64_16x16x4f64.  FP32/BF16 forms: v_mfma_f32_16x16x32_bf16
// with every FP32 operand split into two BF16 terms (x = hi + lo) and the
// three leading products hi*hi + hi*lo + lo*hi accumulated in FP32; spins are
// exact in BF16.
//
// No kernel here uses atomics or fences: every reduction is a fixed-order
// sum of per-block partials done by the consumer kernel (each block of the
// consumer recomputes the same sum), and block 0 publishes the CG scalars for
// the host.
#include "kernels.h"

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

// fixed-order sum of nb partials, identical in every block
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nb, double* sh) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) a += part[b];
    return bsum256(a, sh);
}

__device__ __forceinline__ uint16_t bf16_rn(float f) { return f32_to_bf16_bits(f); }

// x ~= hi + lo in BF16
__device__ __forceinline__ void split2(float x, uint16_t& hi, uint16_t& lo) {
    hi = bf16_rn(x);
    lo = bf16_rn(x - bf16_bits_to_f32(hi));
}

// ---------------------------------------------------------------------------
// per-step layout kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prep_spins(const int8_t* __restrict__ s, int N, long n,
                                                    int Kb, long Nsp, int8_t* __restrict__ Sp,
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
        if (i < Kb) Sp[k * Kb + i] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int il = e >> 6, kl = e & 63;
        const int i = i0 + il;
        if (i < Kb) St[(long)i * Nsp + k0 + kl] = tile[kl][il];
    }
}

template <typename R, int MODE>
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
        if constexpr (MODE == 0) {
            ((double*)out)[o] = (double)tile[kl][jl];
        } else {
            uint16_t hi, lo;
            split2((float)tile[kl][jl], hi, lo);
            ((uint16_t*)out)[o] = hi;
            ((uint16_t*)out)[(size_t)Ma * Nsp + o] = lo;
        }
    }
}

// ---------------------------------------------------------------------------
// CG direction (start of iteration it):
//   rr_it = r.r from the partials of the previous update; stop if
//   rr_it <= tol^2 rr_0, it >= maxiter or non-finite; else beta = rr_it /
//   rr_{it-1} (0 at it = 0) and p_new = r + beta p_old.
// p_new is written in FP64 [Ma][Na] and in the operand layout of
// contraction 1: FP64 path k-major [Kb][Ma]; BF16 forms two planes [Ma][Kb].
// One thread per (j, i < Kb).
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_pnew(Dims d, const double* __restrict__ r,
                                              const double* __restrict__ p_old,
                                              double* __restrict__ p_new, void* __restrict__ Pop,
                                              const double* __restrict__ rrp_cur,
                                              const double* __restrict__ rrp_prev, int nbu, int it,
                                              double tol, int maxiter, CgScalars* sc) {
    if (sc->done) return;
    __shared__ double sh[4];
    const double rr = sum_partials(rrp_cur, nbu, sh);
    const double rrprev = it > 0 ? sum_partials(rrp_prev, nbu, sh) : rr;
    const double rr0 = it == 0 ? rr : sc->rr0;
    const double tol2 = tol * tol * rr0;
    const bool stop = !(rr > tol2) || it >= maxiter || !isfinite(rr);
    const double beta = it == 0 ? 0.0 : rr / rrprev;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rr = rr;
        sc->iters = it;
        sc->beta = beta;
        if (it == 0) {
            sc->rr0 = rr0;
            sc->tol2 = tol2;
        }
        if (stop) {
            sc->done = 1;
            if (!isfinite(rr)) sc->bad = 1;
        }
    }
    if (stop) return;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= d.Ma * d.Kb) return;
    const int j = e / d.Kb, i = e - j * d.Kb;
    double v = 0.0;
    if (i < d.Na) {
        const size_t g = (size_t)j * d.Na + i;
        v = r[g] + beta * p_old[g];
        p_new[g] = v;
    }
    if constexpr (MODE == 0) {
        ((double*)Pop)[(size_t)i * d.Ma + j] = v;
    } else {
        uint16_t hi, lo;
        split2((float)v, hi, lo);
        ((uint16_t*)Pop)[e] = hi;
        ((uint16_t*)Pop)[(size_t)d.Ma * d.Kb + e] = lo;
    }
}

// ---------------------------------------------------------------------------
// contraction 1: w_k = t~_k . (P s~_k) for 16 samples per block; the four
// waves split the hidden tiles (wave w: tiles w, w + 4, ...) and their row
// sums meet in LDS.  Operands come straight from L2: spins from Sp, P in the
// layout written by k_pnew.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_w3(Dims d, const int8_t* __restrict__ Sp,
                                            const void* __restrict__ tact_v, long n,
                                            const void* __restrict__ Pop,
                                            double* __restrict__ w, double* __restrict__ wpart,
                                            const CgScalars* __restrict__ sc) {
    if (sc->done) return;
    __shared__ double wsh[4][16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long r0 = (long)blockIdx.x * 16;
    const int Kb = d.Kb, Ma = d.Ma, nct = d.Ma / 16;
    const int8_t* Srow = Sp + (r0 + lr) * Kb;
    double rs[4] = {0, 0, 0, 0};
    if constexpr (MODE == 0) {
        const double* Pt = (const double*)Pop;
        const double* tact = (const double*)tact_v;
        for (int ct = wave; ct < nct; ct += 4) {
            v4d acc = v4d{0, 0, 0, 0};
            const double* Pc = Pt + ct * 16 + lr;
            for (int k0 = 0; k0 < d.Na; k0 += 4) {
                const double a = (double)Srow[k0 + lk];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Pc[(size_t)(k0 + lk) * Ma], acc, 0, 0, 0);
            }
            const int j = ct * 16 + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const long k = r0 + acc_row<double>(lk, q);
                rs[q] += (k < n ? tact[k * d.Mw + j] : 0.0) * acc[q];
            }
        }
    } else {
        const uint16_t* Ph = (const uint16_t*)Pop;
        const uint16_t* Pl = Ph + (size_t)Ma * Kb;
        const float* tact = (const float*)tact_v;
        float rsf[4] = {0, 0, 0, 0};
        for (int ct = wave; ct < nct; ct += 4) {
            v4f acc = v4f{0, 0, 0, 0};
            const size_t prow = (size_t)(ct * 16 + lr) * Kb + 8 * lk;
            for (int k0 = 0; k0 < Kb; k0 += 32) {
                const uint64_t sb = *(const uint64_t*)(Srow + k0 + 8 * lk);
                v8s av;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int8_t sv = (int8_t)(sb >> (8 * e));
                    av[e] = sv > 0 ? (short)0x3F80 : (sv < 0 ? (short)0xBF80 : (short)0);
                }
                const v8bf a = __builtin_bit_cast(v8bf, av);
                const v8s bh = *(const v8s*)(Ph + prow + k0);
                const v8s bl = *(const v8s*)(Pl + prow + k0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(v8bf, bh), acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(v8bf, bl), acc, 0, 0, 0);
            }
            const int j = ct * 16 + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const long k = r0 + acc_row<float>(lk, q);
                rsf[q] += (k < n ? tact[k * d.Mw + j] : 0.0f) * acc[q];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) rs[q] = (double)rsf[q];
    }
    // row sums over the 16 columns of each tile, then over the four waves
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double v = row16_sum(rs[q]);
        if (lr == 0) wsh[wave][MODE == 0 ? acc_row<double>(lk, q) : acc_row<float>(lk, q)] = v;
    }
    __syncthreads();
    if (tid < 16) {
        const long k = r0 + tid;
        const double v = (wsh[0][tid] + wsh[1][tid]) + (wsh[2][tid] + wsh[3][tid]);
        if (k < n) w[k] = v;
        wsh[0][tid] = k < n ? v : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += wsh[0][q];
        wpart[blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// contraction 2: part[kc][j][i] = sum_{k in chunk kc} t~_kj z_k s~_ki
// v_mode 0: z_k = (w_k - mean w) / n with mean w from the contraction-1
// partials; v_mode 1: z_k = v_k.  grid = (Ma / 16, Nsp / 256): one hidden
// tile and one chunk of 256 samples per block; the tile's t~ rows and the
// chunk's z are staged in LDS and the four waves split the site tiles.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_outer3(Dims d, const int8_t* __restrict__ St,
                                                const void* __restrict__ Th, long Nsp, long n,
                                                const double* __restrict__ v, int v_mode,
                                                const double* __restrict__ wpart, int nbw,
                                                void* __restrict__ part_v,
                                                const CgScalars* __restrict__ sc) {
    if (v_mode == 0 && sc->done) return;
    constexpr int KC = 256;
    __shared__ double sh[4];
    constexpr int KD = KC + 1;  // FP64 row stride: the 16 rows fall in distinct banks
    __shared__ __align__(16) char lds[MODE == 0 ? 16 * KD * 8 + KC * 8 : 2 * 16 * (KC + 8) * 2 + 2 * KC * 2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    double shift = 0.0, scale = 1.0;
    if (v_mode == 0) {
        shift = sum_partials(wpart, nbw, sh) / (double)n;
        scale = 1.0 / (double)n;
    }
    const int jt = blockIdx.x;
    const long kbeg = (long)blockIdx.y * KC;
    const int nit = d.Na / 16;
    if constexpr (MODE == 0) {
        double* As = (double*)lds;           // [16][KD]
        double* zs = As + 16 * KD;           // [KC]
        const double* T = (const double*)Th;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = u * 256 + tid;
            const int rl = e / KC, kl = e - rl * KC;
            As[rl * KD + kl] = T[(size_t)(jt * 16 + rl) * Nsp + kbeg + kl];
        }
        {
            const long k = kbeg + tid;
            zs[tid] = k < n ? (v[k] - shift) * scale : 0.0;
        }
        __syncthreads();
        for (int it = wave; it < nit; it += 4) {
            v4d acc = v4d{0, 0, 0, 0};
            const int8_t* Sr = St + (size_t)(it * 16 + lr) * Nsp + kbeg;
#pragma unroll 2
            for (int k0 = 0; k0 < KC; k0 += 16) {
                const uint32_t sb = *(const uint32_t*)(Sr + k0 + 4 * lk);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int kl = k0 + 4 * lk + e;
                    const int sv = (int8_t)(sb >> (8 * e));
                    const double z = zs[kl];
                    const double b = sv > 0 ? z : (sv < 0 ? -z : 0.0);
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[lr * KD + kl], b, acc, 0, 0, 0);
                }
            }
            double* out = (double*)part_v + (size_t)blockIdx.y * d.Ma * d.Na;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                out[(size_t)(jt * 16 + acc_row<double>(lk, q)) * d.Na + it * 16 + lr] = acc[q];
        }
    } else {
        constexpr int KP = KC + 8;
        uint16_t* Ah = (uint16_t*)lds;       // [16][KP]
        uint16_t* Al = Ah + 16 * KP;
        uint16_t* zh = Al + 16 * KP;         // [KC]
        uint16_t* zl = zh + KC;
        const uint16_t* Thi = (const uint16_t*)Th;
        const uint16_t* Tlo = Thi + (size_t)d.Ma * Nsp;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = u * 256 + tid;
            const int rl = e / KC, kl = e - rl * KC;
            const size_t g = (size_t)(jt * 16 + rl) * Nsp + kbeg + kl;
            Ah[rl * KP + kl] = Thi[g];
            Al[rl * KP + kl] = Tlo[g];
        }
        {
            const long k = kbeg + tid;
            const float z = k < n ? (float)((v[k] - shift) * scale) : 0.0f;
            uint16_t h, l;
            split2(z, h, l);
            zh[tid] = h;
            zl[tid] = l;
        }
        __syncthreads();
        for (int it = wave; it < nit; it += 4) {
            v4f acc = v4f{0, 0, 0, 0};
            const int8_t* Sr = St + (size_t)(it * 16 + lr) * Nsp + kbeg;
#pragma unroll 2
            for (int k0 = 0; k0 < KC; k0 += 32) {
                const int kk = k0 + 8 * lk;
                const v8bf ah = __builtin_bit_cast(v8bf, *(const v8s*)(Ah + lr * KP + kk));
                const v8bf al = __builtin_bit_cast(v8bf, *(const v8s*)(Al + lr * KP + kk));
                const v8s zhv = *(const v8s*)(zh + kk);
                const v8s zlv = *(const v8s*)(zl + kk);
                const uint64_t sb = *(const uint64_t*)(Sr + kk);
                v8s bh, bl;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int8_t sv = (int8_t)(sb >> (8 * e));
                    const short sgn = sv < 0 ? (short)0x8000 : (short)0;
                    bh[e] = sv ? (short)(zhv[e] ^ sgn) : (short)0;
                    bl[e] = sv ? (short)(zlv[e] ^ sgn) : (short)0;
                }
                const v8bf b1 = __builtin_bit_cast(v8bf, bh);
                const v8bf b2 = __builtin_bit_cast(v8bf, bl);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b1, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b2, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b1, acc, 0, 0, 0);
            }
            float* out = (float*)part_v + (size_t)blockIdx.y * d.Ma * d.Na;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                out[(size_t)(jt * 16 + acc_row<float>(lk, q)) * d.Na + it * 16 + lr] = acc[q];
        }
    }
}

// out[e] = sum_kc part[kc][e] + shift p[e] (parameter entries only); with p,
// also the block partials of p . out.
template <typename R>
__global__ __launch_bounds__(256) void k_reduce2(Dims d, const R* __restrict__ part, int ksplit,
                                                 const double* __restrict__ p, double shift,
                                                 double* __restrict__ out,
                                                 double* __restrict__ pap,
                                                 const CgScalars* __restrict__ sc, int cg) {
    if (cg && sc->done) return;
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
            for (; kc + 16 <= ksplit; kc += 16) {
                R x[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) x[u] = part[(size_t)(kc + u) * total + e];
#pragma unroll
                for (int u = 0; u < 16; ++u) val += (double)x[u];
            }
            for (; kc < ksplit; ++kc) val += (double)part[(size_t)kc * total + e];
            if (p) val += shift * p[e];
        }
        out[e] = val;
        if (p) dot = val * p[e];
    }
    if (!cg) return;
    dot = bsum256(dot, sh);
    if (threadIdx.x == 0) pap[blockIdx.x] = dot;
}

// alpha = rr / p.Ap; x += alpha p; r -= alpha Ap; block partials of r.r.
__global__ __launch_bounds__(256) void k_update2(int total, double* __restrict__ x,
                                                 double* __restrict__ r,
                                                 const double* __restrict__ p,
                                                 const double* __restrict__ Ap,
                                                 const double* __restrict__ pap, int nbr,
                                                 const double* __restrict__ rrp_cur,
                                                 double* __restrict__ rrp_next, int nbu,
                                                 CgScalars* sc) {
    if (sc->done) return;
    __shared__ double sh[4];
    const double pAp = sum_partials(pap, nbr, sh);
    const double rr = sum_partials(rrp_cur, nbu, sh);
    const double alpha = rr / pAp;
    if (!(pAp > 0.0) || !isfinite(alpha)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->bad = 1;
            sc->done = 1;
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->alpha = alpha;
        sc->pAp = pAp;
    }
    const int e = blockIdx.x * 256 + threadIdx.x;
    double q = 0.0;
    if (e < total) {
        x[e] += alpha * p[e];
        const double re = r[e] - alpha * Ap[e];
        r[e] = re;
        q = re * re;
    }
    q = bsum256(q, sh);
    if (threadIdx.x == 0) rrp_next[blockIdx.x] = q;
}

// x = 0, r = p = f, partials of f.f; clears the CG flags.
__global__ __launch_bounds__(256) void k_init2(int total, const double* __restrict__ f,
                                               double* __restrict__ x, double* __restrict__ r,
                                               double* __restrict__ p, double* __restrict__ rrp0,
                                               CgScalars* sc) {
    __shared__ double sh[4];
    const int e = blockIdx.x * 256 + threadIdx.x;
    double q = 0.0;
    if (e < total) {
        const double fe = f[e];
        x[e] = 0.0;
        r[e] = fe;
        p[e] = fe;
        q = fe * fe;
    }
    q = bsum256(q, sh);
    if (threadIdx.x == 0) rrp0[blockIdx.x] = q;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->done = 0;
        sc->bad = 0;
        sc->iters = 0;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int nb_of(long n, int b) { return (int)((n + b - 1) / b); }

long qgt_padded_samples(long n) { return (n + 255) / 256 * 256; }

size_t qgt_th_bytes(const Dims& d, int prec, long Nsp) {
    return (size_t)d.Ma * Nsp * (prec == 0 ? 8 : 4);
}

void launch_qgt_prepare(hipStream_t st, const Dims& d, int prec, const int8_t* s,
                        const void* tact, long n, const QgtBatch& q) {
    const dim3 gs((unsigned)(q.Nsp / 64), (unsigned)nb_of(d.Kb, 64));
    k_prep_spins<<<gs, 256, 0, st>>>(s, d.N, n, d.Kb, q.Nsp, q.Sp, q.St);
    const dim3 gt((unsigned)(q.Nsp / 64), (unsigned)nb_of(d.Ma, 64));
    if (prec == 0)
        k_prep_t<double, 0><<<gt, 256, 0, st>>>((const double*)tact, n, d.Mw, d.Ma, q.Nsp, q.Th);
    else
        k_prep_t<float, 1><<<gt, 256, 0, st>>>((const float*)tact, n, d.Mw, d.Ma, q.Nsp, q.Th);
}

int qgt_nbw(long n) { return nb_of(n, 16); }
int qgt_nbu(const Dims& d) { return nb_of((long)d.Ma * d.Na, 256); }
size_t qgt_pop_bytes(const Dims& d, int prec) {
    return prec == 0 ? (size_t)d.Kb * d.Ma * 8 : (size_t)2 * d.Ma * d.Kb * 2;
}

void launch_qgt_pnew(hipStream_t st, const Dims& d, int prec, const double* r,
                     const double* p_old, double* p_new, void* Pop, const double* rrp_cur,
                     const double* rrp_prev, int it, double tol, int maxiter, CgScalars* sc) {
    const int nb = nb_of((long)d.Ma * d.Kb, 256), nbu = qgt_nbu(d);
    if (prec == 0)
        k_pnew<0><<<nb, 256, 0, st>>>(d, r, p_old, p_new, Pop, rrp_cur, rrp_prev, nbu, it, tol,
                                      maxiter, sc);
    else
        k_pnew<1><<<nb, 256, 0, st>>>(d, r, p_old, p_new, Pop, rrp_cur, rrp_prev, nbu, it, tol,
                                      maxiter, sc);
}

void launch_qgt_w(hipStream_t st, const Dims& d, int prec, const QgtBatch& q, const void* tact,
                  long n, const void* Pop, double* w, const CgScalars* sc) {
    const int nb = qgt_nbw(n);
    if (prec == 0)
        k_w3<0><<<nb, 256, 0, st>>>(d, q.Sp, tact, n, Pop, w, q.wpart, sc);
    else
        k_w3<1><<<nb, 256, 0, st>>>(d, q.Sp, tact, n, Pop, w, q.wpart, sc);
}

int qgt_ksplit(const QgtBatch& q) { return (int)(q.Nsp / 256); }

void launch_qgt_outer(hipStream_t st, const Dims& d, int prec, const QgtBatch& q, long n,
                      const double* v, int v_mode, void* part, const CgScalars* sc) {
    const dim3 grid((unsigned)(d.Ma / 16), (unsigned)qgt_ksplit(q));
    const int nbw = qgt_nbw(n);
    if (prec == 0)
        k_outer3<0><<<grid, 256, 0, st>>>(d, q.St, q.Th, q.Nsp, n, v, v_mode, q.wpart, nbw, part,
                                         sc);
    else
        k_outer3<1><<<grid, 256, 0, st>>>(d, q.St, q.Th, q.Nsp, n, v, v_mode, q.wpart, nbw, part,
                                         sc);
}

void launch_qgt_reduce(hipStream_t st, const Dims& d, int prec, const void* part, int ksplit,
                       const double* p, double shift, double* out, double* pap,
                       const CgScalars* sc, int cg) {
    const int nb = qgt_nbu(d);
    if (prec == 0)
        k_reduce2<double><<<nb, 256, 0, st>>>(d, (const double*)part, ksplit, p, shift, out, pap,
                                              sc, cg);
    else
        k_reduce2<float><<<nb, 256, 0, st>>>(d, (const float*)part, ksplit, p, shift, out, pap,
                                             sc, cg);
}

void launch_qgt_update(hipStream_t st, const Dims& d, double* x, double* r, const double* p,
                       const double* Ap, const double* pap, const double* rrp_cur,
                       double* rrp_next, CgScalars* sc) {
    const int nb = qgt_nbu(d);
    k_update2<<<nb, 256, 0, st>>>(d.Ma * d.Na, x, r, p, Ap, pap, nb, rrp_cur, rrp_next, nb, sc);
}

void launch_qgt_init(hipStream_t st, const Dims& d, const double* f, double* x, double* r,
                     double* p, double* rrp0, CgScalars* sc) {
    const int nb = qgt_nbu(d);
    k_init2<<<nb, 256, 0, st>>>(d.Ma * d.Na, f, x, r, p, rrp0, sc);
}

}  // namespace nqs
