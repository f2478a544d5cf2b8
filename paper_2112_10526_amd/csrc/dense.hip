// Dense-Jacobian form of the QGT (paper, QGTJacobianDense and its appendix):
// the Jacobian O[k][p] = d ln psi(s_k) / d p_p is materialised in the packed
// parameter order, centred and scaled (dJ = (O - mean O) / sqrt(N_s)), the
// Gram matrix G = dJ^T dJ is formed on MFMA, and CG runs on G v + eps v.
#include "kernels.h"

#include <vector>

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
// Column sums in two fixed-order passes: `splits` slices of rows give partial
// sums (one thread per column and slice), then each column adds its slices in
// order.  Then O <- (O - colsum / n) / sqrt(n), four columns per thread where
// the rows are 16-byte aligned.
constexpr int CS_SPLIT_MAX = 64;
template <typename R>
__global__ __launch_bounds__(256) void k_colsum_part(const R* __restrict__ O, long n, long ld,
                                                     int P, int splits, double* __restrict__ part) {
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const long k0 = n * blockIdx.y / splits, k1 = n * (blockIdx.y + 1) / splits;
    double acc = 0.0;
    for (long k = k0; k < k1; ++k) acc += (double)O[k * ld + p];
    part[(size_t)blockIdx.y * P + p] = acc;
}
__global__ __launch_bounds__(256) void k_colsum_fin(const double* __restrict__ part, int P,
                                                    int splits, double* __restrict__ cs) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    double acc = 0.0;
    for (int q = 0; q < splits; ++q) acc += part[(size_t)q * P + p];
    cs[p] = acc;
}
// SPLIT (FP32 entries, dense form of the BF16 precision): each centred entry x
// is stored in its own 4 bytes as the BF16 pair (hi << 16) | lo, hi = bf16(x),
// lo = bf16(x - hi), the operand form of the BF16 Gram.
template <typename R, bool SPLIT>
__device__ __forceinline__ R center_store(double v) {
    if constexpr (SPLIT) {
        const float x = (float)v;
        const uint16_t hi = f32_to_bf16_bits(x);
        const uint16_t lo = f32_to_bf16_bits(x - bf16_bits_to_f32(hi));
        return __builtin_bit_cast(float, ((uint32_t)hi << 16) | lo);
    } else {
        return (R)v;
    }
}
template <typename R, bool SPLIT = false>
__global__ __launch_bounds__(256) void k_center_scale(R* __restrict__ O, long n, long ld, int P,
                                                      const double* __restrict__ cs, int vec) {
    const long k = blockIdx.y;
    const int W = vec ? 4 : 1;  // columns per thread
    const long p = W * ((long)blockIdx.x * 256 + threadIdx.x);
    if (p >= P || k >= n) return;
    const double inv = 1.0 / (double)n;
    const double rs = 1.0 / sqrt((double)n);
    R* e = O + k * ld + p;
    if (vec && p + 4 <= P) {  // (ld a multiple of 4, base 16-byte aligned, p a multiple of 4)
        if constexpr (sizeof(R) == 4) {
            float4 t = *(float4*)e;
            t.x = center_store<R, SPLIT>(((double)t.x - cs[p] * inv) * rs);
            t.y = center_store<R, SPLIT>(((double)t.y - cs[p + 1] * inv) * rs);
            t.z = center_store<R, SPLIT>(((double)t.z - cs[p + 2] * inv) * rs);
            t.w = center_store<R, SPLIT>(((double)t.w - cs[p + 3] * inv) * rs);
            *(float4*)e = t;
        } else {
            double2 a = *(double2*)e, b = *(double2*)(e + 2);
            a.x = (a.x - cs[p] * inv) * rs;
            a.y = (a.y - cs[p + 1] * inv) * rs;
            b.x = (b.x - cs[p + 2] * inv) * rs;
            b.y = (b.y - cs[p + 3] * inv) * rs;
            *(double2*)e = a;
            *(double2*)(e + 2) = b;
        }
    } else {
        for (long q = p; q < P && q < p + W; ++q)
            e[q - p] = center_store<R, SPLIT>(((double)e[q - p] - cs[q] * inv) * rs);
    }
}

// The Jacobian's entries straight from a sample's spins and activations: the
// entry of column p is s_i (visible bias), t_j (hidden bias) or t_j s_i (W_ji),
// with the packed order [a | b | W] and W row-major (p = off + j N + i); t_j s_i
// with s_i = +-1 is exact in FP32, so it is the stored entry's value.
struct JacCol {
    int kind, j, i;  // kind 0: s_i, 1: t_j, 2: t_j s_i, 3: padding (zero)
};
__device__ __forceinline__ JacCol jac_col(const Dims& d, long p, int P) {
    JacCol c{3, 0, 0};
    if (p >= P) return c;
    long idx = p;
    if (d.vb) {
        if (idx < d.N) return JacCol{0, 0, (int)idx};
        idx -= d.N;
    }
    if (d.hb) {
        if (idx < d.M) return JacCol{1, (int)idx, 0};
        idx -= d.M;
    }
    const int j = (int)(idx / d.N);
    return JacCol{2, j, (int)(idx - (long)j * d.N)};
}
// Column sums over the same row slices, in the same order, as k_colsum_part,
// read from the spins and activations instead of a materialised Jacobian.  A
// missing factor (the spin of a hidden-bias column, the activation of a
// visible-bias column) is read as the constant 1 with stride 0, so the loop has
// no branch; 1 * x is x exactly, so the sums are unchanged.
__device__ const int8_t k_one_s = 1;
template <typename R>
__device__ const R k_one_t = (R)1;
template <typename R>
__global__ __launch_bounds__(256) void k_colsum_st(Dims d, const int8_t* __restrict__ s,
                                                   const R* __restrict__ tact, long n, int P,
                                                   int splits, double* __restrict__ part) {
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const JacCol c = jac_col(d, p, P);
    const bool has_s = c.kind != 1, has_t = c.kind != 0;
    const int8_t* sp = has_s ? s + c.i : &k_one_s;
    const R* tp = has_t ? tact + c.j : &k_one_t<R>;
    const long ss = has_s ? d.N : 0, ts = has_t ? d.Mw : 0;
    const long k0 = n * blockIdx.y / splits, k1 = n * (blockIdx.y + 1) / splits;
    double acc = 0.0;
    long k = k0;
    for (; k + 4 <= k1; k += 4) {  // (loads of four rows issued together; sum order unchanged)
        const double t0 = (double)tp[k * ts], t1 = (double)tp[(k + 1) * ts];
        const double t2 = (double)tp[(k + 2) * ts], t3 = (double)tp[(k + 3) * ts];
        const double s0 = (double)sp[k * ss], s1 = (double)sp[(k + 1) * ss];
        const double s2 = (double)sp[(k + 2) * ss], s3 = (double)sp[(k + 3) * ss];
        acc += t0 * s0;
        acc += t1 * s1;
        acc += t2 * s2;
        acc += t3 * s3;
    }
    for (; k < k1; ++k) acc += (double)tp[k * ts] * (double)sp[k * ss];
    part[(size_t)blockIdx.y * P + p] = acc;
}

// Centred, scaled Jacobian written in one pass: dJ[k][p] = (O[k][p] - cs[p] / n)
// / sqrt(n) (the same expression as k_center_scale over a materialised O), zero
// in the padding columns P <= p < ld.  Four columns per thread, JC_ROWS rows per
// block; vec: ld a multiple of 4 and O 16-byte aligned (one 16-byte store per
// FP32 row, two per FP64 row).  Each column reads its spin and activation through
// a pointer and a row stride, a missing factor being the constant 1 (or 0 for
// padding) with stride 0, so a full block of rows issues all its loads before
// any arithmetic.
__device__ const int8_t k_zero_s = 0;
constexpr int JC_ROWS = 8;
template <typename R, bool SPLIT>
__global__ __launch_bounds__(256) void k_jacobian_centred(Dims d, const int8_t* __restrict__ s,
                                                          const R* __restrict__ tact, long n,
                                                          long rows, int P, long ld,
                                                          const double* __restrict__ cs, int vec,
                                                          R* __restrict__ O) {
    const long p = 4 * ((long)blockIdx.x * 256 + threadIdx.x);
    if (p >= ld) return;
    const double inv = 1.0 / (double)n;  // (n: all samples; rows: this launch's)
    const double rs = 1.0 / sqrt((double)n);
    const int8_t* sp[4];
    const R* tp[4];
    long ss[4], ts[4];
    double mean[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const JacCol c = jac_col(d, p + e, P);
        const bool has_s = c.kind == 0 || c.kind == 2, has_t = c.kind == 1 || c.kind == 2;
        sp[e] = has_s ? s + c.i : (c.kind == 3 ? &k_zero_s : &k_one_s);
        ss[e] = has_s ? d.N : 0;
        tp[e] = has_t ? tact + c.j : &k_one_t<R>;
        ts[e] = has_t ? d.Mw : 0;
        mean[e] = c.kind != 3 ? cs[p + e] * inv : 0.0;
    }
    const long k0 = (long)blockIdx.y * JC_ROWS;
    auto store = [&](long k, const double* x) {
        R v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = center_store<R, SPLIT>((x[e] - mean[e]) * rs);
        R* row = O + k * ld + p;
        if (vec) {
            if constexpr (sizeof(R) == 4) {
                *(float4*)row = make_float4(v[0], v[1], v[2], v[3]);
            } else {
                *(double2*)row = make_double2(v[0], v[1]);
                *(double2*)(row + 2) = make_double2(v[2], v[3]);
            }
        } else {
            for (int e = 0; e < 4 && p + e < ld; ++e) row[e] = v[e];
        }
    };
    if (k0 + JC_ROWS <= rows) {
        double x[JC_ROWS][4];
#pragma unroll
        for (int r = 0; r < JC_ROWS; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                x[r][e] = (double)tp[e][(k0 + r) * ts[e]] * (double)sp[e][(k0 + r) * ss[e]];
#pragma unroll
        for (int r = 0; r < JC_ROWS; ++r) store(k0 + r, x[r]);
    } else {
        for (long k = k0; k < rows; ++k) {
            double x[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) x[e] = (double)tp[e][k * ts[e]] * (double)sp[e][k * ss[e]];
            store(k, x);
        }
    }
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

// FP64 Gram over row slices, for matrices with few tiles (a small P leaves most
// compute units idle when each tile walks all n rows): block = (tile, slice of
// rows), the tile's partial written in tile order [128][128]; k_gram_fin sums
// the slices in order (deterministic) and writes G with the lower triangle
// mirrored (within a diagonal tile only entries on or above the diagonal are
// taken, so G is exactly symmetric).
__global__ __launch_bounds__(256) void k_gram_slices(const double* __restrict__ A, long n, long ld,
                                                     int ntiles, long rows_per_slice,
                                                     const int* __restrict__ tiles,
                                                     double* __restrict__ part) {
    const int t = (int)(blockIdx.x % (unsigned)ntiles), ks = (int)(blockIdx.x / (unsigned)ntiles);
    const int tp = tiles[2 * t], tq = tiles[2 * t + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long p0 = (long)tp * 128 + (wave >> 1) * 64;
    const long q0 = (long)tq * 128 + (wave & 1) * 64;
    const long r0 = (long)ks * rows_per_slice;
    const long r1 = r0 + rows_per_slice < n ? r0 + rows_per_slice : n;
    v4d acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0, 0, 0, 0};
    for (long k0 = r0; k0 < r1; k0 += 4) {
        const long k = k0 + lk;
        double fa[4], fb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            fa[a] = k < r1 ? A[k * ld + p0 + a * 16 + lr] : 0.0;
            fb[a] = k < r1 ? A[k * ld + q0 + a * 16 + lr] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    double* pt = part + (size_t)blockIdx.x * 128 * 128;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int pr = (wave >> 1) * 64 + a * 16 + acc_row<double>(lk, i);
                const int qc = (wave & 1) * 64 + b * 16 + lr;
                pt[pr * 128 + qc] = acc[a][b][i];
            }
}

__global__ __launch_bounds__(256) void k_gram_fin(const double* __restrict__ part, int ntiles,
                                                  int slices, const int* __restrict__ tiles, int P,
                                                  long ld, double* __restrict__ G) {
    __shared__ double sg[32][33];
    const int t = blockIdx.x >> 4, sub = blockIdx.x & 15;
    const int tp = tiles[2 * t], tq = tiles[2 * t + 1];
    const int i0 = (sub >> 2) * 32, j0 = (sub & 3) * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const long P0 = (long)tp * 128, Q0 = (long)tq * 128;
    const bool diag = tp == tq;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int ii = ty + 8 * m, jj = tx;
        const size_t e = (size_t)(i0 + ii) * 128 + (j0 + jj);
        double a = 0.0;
        for (int ks = 0; ks < slices; ++ks) a += part[((size_t)ks * ntiles + t) * 128 * 128 + e];
        sg[ii][jj] = a;
        const long p = P0 + i0 + ii, q = Q0 + j0 + jj;
        if ((!diag || i0 + ii <= j0 + jj) && p < P && q < P) G[p * ld + q] = a;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int jj = ty + 8 * m, ii = tx;  // element (ii, jj) written at (q, p)
        const long p = P0 + i0 + ii, q = Q0 + j0 + jj;
        if ((!diag || i0 + ii < j0 + jj) && p < P && q < P) G[q * ld + p] = sg[ii][jj];
    }
}

// BF16 form: the same Gram on the BF16 matrix cores.  The centring kernel has
// stored every entry x as the BF16 pair (hi << 16) | lo with x ~= hi + lo;
// three products (hi hi + hi lo + lo hi) are accumulated in FP32: about 2^-16
// relative error per product at BF16 rates.  A slice of GS_K samples of the
// block's two 128-column panels is loaded (each thread: 4 consecutive samples x
// 4 consecutive columns of each panel, 16 bytes per sample), regrouped into
// hi and lo planes and stored in LDS transposed ([column][sample], the
// contracted index contiguous for the MFMA operands, 4 samples per 8-byte
// store); the next slice's loads are issued before the current slice's MFMAs.
constexpr int GS_K = 32, GS_KP = GS_K + 8;  // samples per slice; LDS row stride (halves)
typedef short v8s_g __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(256) void k_gram_split(const uint32_t* __restrict__ A, long n, long ld,
                                                    int P, float* __restrict__ G,
                                                    const int* __restrict__ tiles) {
    __shared__ __align__(16) uint16_t Ls[2][2][128 * GS_KP];  // [panel p/q][hi/lo][col][sample]
    const int tp = tiles[2 * blockIdx.x], tq = tiles[2 * blockIdx.x + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long base[2] = {(long)tp * 128, (long)tq * 128};
    const int rg = tid & 7, c4 = tid >> 3;  // rows 4 rg .. 4 rg + 3, columns 4 c4 .. 4 c4 + 3
    uint4 ra[2][4];
    auto load = [&](long k0) {
#pragma unroll
        for (int op = 0; op < 2; ++op)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const long k = k0 + 4 * rg + j;
                ra[op][j] = k < n ? *(const uint4*)(A + k * ld + base[op] + 4 * c4)
                                  : make_uint4(0u, 0u, 0u, 0u);
            }
    };
    auto stage = [&]() {
#pragma unroll
        for (int op = 0; op < 2; ++op)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                uint32_t w[4];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    w[j] = e == 0 ? ra[op][j].x : e == 1 ? ra[op][j].y : e == 2 ? ra[op][j].z : ra[op][j].w;
                // samples (j, j + 1) -> one word per plane, the earlier sample in the low half
                const uint2 hi = make_uint2((w[1] & 0xFFFF0000u) | (w[0] >> 16),
                                            (w[3] & 0xFFFF0000u) | (w[2] >> 16));
                const uint2 lo = make_uint2((w[1] << 16) | (w[0] & 0xFFFFu),
                                            (w[3] << 16) | (w[2] & 0xFFFFu));
                const int off = (4 * c4 + e) * GS_KP + 4 * rg;
                *(uint2*)&Ls[op][0][off] = hi;
                *(uint2*)&Ls[op][1][off] = lo;
            }
    };
    v4f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0, 0, 0, 0};
    const int pr = (wave >> 1) * 64, qr = (wave & 1) * 64;  // the wave's quarter
    load(0);
    for (long k0 = 0; k0 < n; k0 += GS_K) {
        __syncthreads();  // the previous slice is no longer read
        stage();
        __syncthreads();
        if (k0 + GS_K < n) load(k0 + GS_K);
        v8s_g ah[4], al[4], bh[4], bl[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int cp = (pr + a * 16 + lr) * GS_KP + 8 * lk;
            const int cq = (qr + a * 16 + lr) * GS_KP + 8 * lk;
            ah[a] = *(const v8s_g*)&Ls[0][0][cp];
            al[a] = *(const v8s_g*)&Ls[0][1][cp];
            bh[a] = *(const v8s_g*)&Ls[1][0][cq];
            bl[a] = *(const v8s_g*)&Ls[1][1][cq];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const v8bf xh = __builtin_bit_cast(v8bf, ah[a]), xl = __builtin_bit_cast(v8bf, al[a]);
                const v8bf yh = __builtin_bit_cast(v8bf, bh[b]), yl = __builtin_bit_cast(v8bf, bl[b]);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yh, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yl, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, yh, acc[a][b], 0, 0, 0);
            }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long p = base[0] + pr + a * 16 + acc_row<float>(lk, i);
                const long q = base[1] + qr + b * 16 + lr;
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

// out = G v + shift v (FP64 accumulation) and the block partials of v . out.
// Each wave handles DMV_RW rows at once, so every 4-element slice of v it loads
// serves DMV_RW rows of G (4 consecutive entries per lane per step).  No
// cross-block step: the CG update sums the partials.
constexpr int DMV_RW = 4;
template <typename R>
__global__ __launch_bounds__(256) void k_dense_matvec(const R* __restrict__ G, int P, long ld,
                                                      const double* __restrict__ v,
                                                      double* __restrict__ out,
                                                      double* __restrict__ dpart,
                                                      const CgScalars* __restrict__ sc) {
    if (sc->done) return;
    __shared__ double sh[4];
    const double shift = sc->shift;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long p0 = ((long)blockIdx.x * 4 + wave) * DMV_RW;
    double acc[DMV_RW];
#pragma unroll
    for (int r = 0; r < DMV_RW; ++r) acc[r] = 0.0;
    for (long q = 4 * lane; q < P; q += 256) {
        if (q + 4 <= P) {
            const double2 v01 = *(const double2*)(v + q), v23 = *(const double2*)(v + q + 2);
#pragma unroll
            for (int r = 0; r < DMV_RW; ++r) {
                if (p0 + r >= P) break;
                const R* g = G + (p0 + r) * ld + q;
                double g0, g1, g2, g3;
                if constexpr (sizeof(R) == 4) {
                    const float4 t = *(const float4*)g;
                    g0 = t.x; g1 = t.y; g2 = t.z; g3 = t.w;
                } else {
                    const double2 a = *(const double2*)g, b = *(const double2*)(g + 2);
                    g0 = a.x; g1 = a.y; g2 = b.x; g3 = b.y;
                }
                acc[r] += (g0 * v01.x + g1 * v01.y) + (g2 * v23.x + g3 * v23.y);
            }
        } else {  // ragged end of the row
            for (long qq = q; qq < P; ++qq)
#pragma unroll
                for (int r = 0; r < DMV_RW; ++r)
                    if (p0 + r < P) acc[r] += (double)G[(p0 + r) * ld + qq] * v[qq];
        }
    }
    double dot = 0.0;
#pragma unroll
    for (int r = 0; r < DMV_RW; ++r) {
        const double s = wave_sum(acc[r]);
        if (p0 + r < P) {
            const double o = s + shift * v[p0 + r];
            if (lane == 0) out[p0 + r] = o;
            dot += o * v[p0 + r];
        }
    }
    if (lane == 0) sh[wave] = dot;
    __syncthreads();
    if (threadIdx.x == 0) dpart[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

int dense_matvec_blocks(int P) { return (P + 4 * DMV_RW - 1) / (4 * DMV_RW); }

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

void launch_center_cols(hipStream_t st, int prec, void* O, long n, long ld, int P, double* cs,
                        double* scratch, size_t scratch_bytes, bool split) {
    const int nb = (P + 255) / 256;
    size_t sp = scratch ? scratch_bytes / (8 * (size_t)P) : 1;
    const int splits = (int)(sp < 1 ? 1 : (sp > CS_SPLIT_MAX ? CS_SPLIT_MAX : sp));
    double* part = splits > 1 ? scratch : cs;  // one slice: the sums go straight to cs
    const dim3 g1(nb, splits);
    const int vec = (ld % 4 == 0 && ((uintptr_t)O & 15) == 0) ? 1 : 0;
    const dim3 g2(vec ? (P + 1023) / 1024 : nb, (unsigned)n);
    if (prec == 0)
        k_colsum_part<double><<<g1, 256, 0, st>>>((const double*)O, n, ld, P, splits, part);
    else
        k_colsum_part<float><<<g1, 256, 0, st>>>((const float*)O, n, ld, P, splits, part);
    if (splits > 1) k_colsum_fin<<<nb, 256, 0, st>>>(part, P, splits, cs);
    if (prec == 0)
        k_center_scale<double><<<g2, 256, 0, st>>>((double*)O, n, ld, P, cs, vec);
    else if (split)
        k_center_scale<float, true><<<g2, 256, 0, st>>>((float*)O, n, ld, P, cs, vec);
    else
        k_center_scale<float><<<g2, 256, 0, st>>>((float*)O, n, ld, P, cs, vec);
}

// Centred, scaled Jacobian of n samples in one write pass (column sums from the
// spins and activations first; scratch holds the slice partials).
void launch_jacobian_centred(hipStream_t st, const Dims& d, int prec, const int8_t* s,
                             const void* tact, long n, void* O, int P, long ld, double* cs,
                             double* scratch, size_t scratch_bytes, bool split) {
    if (n <= 0) return;
    const int nb = (P + 255) / 256;
    size_t sp = scratch ? scratch_bytes / (8 * (size_t)P) : 1;
    const int splits = (int)(sp < 1 ? 1 : (sp > CS_SPLIT_MAX ? CS_SPLIT_MAX : sp));
    double* part = splits > 1 ? scratch : cs;
    const dim3 g1(nb, splits);
    if (prec == 0)
        k_colsum_st<double><<<g1, 256, 0, st>>>(d, s, (const double*)tact, n, P, splits, part);
    else
        k_colsum_st<float><<<g1, 256, 0, st>>>(d, s, (const float*)tact, n, P, splits, part);
    if (splits > 1) k_colsum_fin<<<nb, 256, 0, st>>>(part, P, splits, cs);
    const int vec = (ld % 4 == 0 && ((uintptr_t)O & 15) == 0) ? 1 : 0;
    const size_t es = prec == 0 ? 8 : 4;
    const long chunk = 65535L * JC_ROWS;  // rows per launch (grid y limit)
    for (long r0 = 0; r0 < n; r0 += chunk) {
        const long m = n - r0 < chunk ? n - r0 : chunk;
        const dim3 g2((unsigned)((ld + 1023) / 1024), (unsigned)((m + JC_ROWS - 1) / JC_ROWS));
        const int8_t* sr = s + r0 * d.N;
        const char* tr = (const char*)tact + es * (size_t)r0 * d.Mw;
        char* orow = (char*)O + es * (size_t)r0 * ld;
        if (prec == 0)
            k_jacobian_centred<double, false><<<g2, 256, 0, st>>>(
                d, sr, (const double*)tr, n, m, P, ld, cs, vec, (double*)orow);
        else if (split)
            k_jacobian_centred<float, true><<<g2, 256, 0, st>>>(
                d, sr, (const float*)tr, n, m, P, ld, cs, vec, (float*)orow);
        else
            k_jacobian_centred<float, false><<<g2, 256, 0, st>>>(
                d, sr, (const float*)tr, n, m, P, ld, cs, vec, (float*)orow);
    }
}

int gram_tiles(int P) {
    const int nt = (P + 127) / 128;
    return nt * (nt + 1) / 2;
}
// Tile order, XCD-aware.  The hardware deals consecutive blocks to the 8 XCDs
// in turn, so block 8 i + e runs on XCD e.  The upper block triangle is cut into
// GT_SUPER x GT_SUPER supertiles, dealt to the XCDs in turn; each XCD runs its
// supertiles one after the other, so the blocks resident on one XCD at a time
// (about 64) share GT_SUPER row panels and GT_SUPER column panels in its L2
// instead of each streaming a panel of its own.  Every tile appears once; the
// ragged end (XCDs with fewer tiles) is filled in order.
constexpr int GT_XCD = 8, GT_SUPER = 8;
void fill_gram_tiles(int P, int* host_tiles) {
    const int nt = (P + 127) / 128, ns = (nt + GT_SUPER - 1) / GT_SUPER;
    std::vector<std::vector<int>> seq(GT_XCD);
    int sid = 0;
    for (int A = 0; A < ns; ++A)
        for (int B = A; B < ns; ++B, ++sid) {
            std::vector<int>& q = seq[sid % GT_XCD];
            for (int a = A * GT_SUPER; a < (A + 1) * GT_SUPER && a < nt; ++a)
                for (int b = B * GT_SUPER; b < (B + 1) * GT_SUPER && b < nt; ++b)
                    if (b >= a) {
                        q.push_back(a);
                        q.push_back(b);
                    }
        }
    size_t pos[GT_XCD] = {0};
    const long total = (long)nt * (nt + 1) / 2;
    long e = 0;
    while (e < total) {  // slot e goes to XCD e % 8 while that XCD has tiles left
        int src = (int)(e % GT_XCD);
        for (int tries = 0; tries < GT_XCD && pos[src] >= seq[src].size(); ++tries)
            src = (src + 1) % GT_XCD;
        host_tiles[2 * e] = seq[src][pos[src]];
        host_tiles[2 * e + 1] = seq[src][pos[src] + 1];
        pos[src] += 2;
        ++e;
    }
}
// Row slices for the FP64 Gram: enough (tile, slice) blocks for two per compute
// unit, each slice at least 128 rows; 1 = the unsliced kernel.
int gram_slices(int ntiles, long n) {
    int S = 1;
    while (S < 256 && (long)ntiles * S < 512 && n / (2 * S) >= 128) S *= 2;
    return S;
}
size_t gram_part_bytes(int ntiles, int slices) {
    return slices > 1 ? (size_t)ntiles * slices * 128 * 128 * 8 : 0;
}
void launch_gram_sliced(hipStream_t st, const double* A, long n, long ld, int P, double* G,
                        const int* tiles, int ntiles, int slices, double* part) {
    if (slices <= 1 || !part) {
        k_gram<double><<<ntiles, 256, 0, st>>>(A, n, ld, P, G, tiles);
        return;
    }
    long rps = (n + slices - 1) / slices;
    rps = (rps + 3) / 4 * 4;
    k_gram_slices<<<(unsigned)(ntiles * slices), 256, 0, st>>>(A, n, ld, ntiles, rps, tiles, part);
    k_gram_fin<<<(unsigned)(ntiles * 16), 256, 0, st>>>(part, ntiles, slices, tiles, P, ld, G);
}
void launch_gram(hipStream_t st, int prec, const void* A, long n, long ld, int P, void* G,
                 const int* tiles, int ntiles) {
    if (prec == 0)
        k_gram<double><<<ntiles, 256, 0, st>>>((const double*)A, n, ld, P, (double*)G, tiles);
    else if (prec == 1)
        k_gram<float><<<ntiles, 256, 0, st>>>((const float*)A, n, ld, P, (float*)G, tiles);
    else  // (split pairs from the centring; ld a multiple of 128: panel loads stay in their row)
        k_gram_split<<<ntiles, 256, 0, st>>>((const uint32_t*)A, n, ld, P, (float*)G, tiles);
}
void launch_dense_matvec(hipStream_t st, int prec, const void* G, int P, long ld, const double* v,
                         double* out, double* dpart, CgScalars* sc) {
    const int nb = dense_matvec_blocks(P);
    if (prec == 0)
        k_dense_matvec<double><<<nb, 256, 0, st>>>((const double*)G, P, ld, v, out, dpart, sc);
    else
        k_dense_matvec<float><<<nb, 256, 0, st>>>((const float*)G, P, ld, v, out, dpart, sc);
}

}  // namespace nqs
