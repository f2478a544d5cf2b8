// Complex-parameter RBM with a holomorphic mapping theta -> psi (paper:
// complex parameters of holomorphic architectures; log-derivative, force and
// QGT estimator equations; complex co-gradient and SR equations; TDVP
// equation of motion), in complex FP64 (double2 = real, imaginary).
//
// Parameters, packed: [a (N) | b (M) | W (M x N), W[j][i] couples hidden j and
// site i].  Tables built from them: T[i][j] = tanh(2 W_ji) (site-major) and the
// site factors K[i] = (K_i(+1), K_i(-1)), K_i(s) = exp(-2 a_i s) prod_j cosh(2 W_ji),
// so that flipping site i of s multiplies psi by
//   K_i(s_i) prod_j (1 - s_i tanh(theta_j) T[i][j])
// (cosh(theta - 2 s W) = cosh(theta) cosh(2W) (1 - s tanh(theta) tanh(2W))).
//
// The dense holomorphic QGT G = dJ^H dJ (dJ = (O - mean O) / sqrt(N_s)) and the
// system (G + eps I) x = f are solved over the reals.  With X = Re dJ, Z = Im dJ,
//   G = A + i B,  A = X^T X + Z^T Z (symmetric),  B = X^T Z - Z^T X (antisymmetric),
// and the real system [[A, -B], [B, A]] [Re x; Im x] = [Re f; Im f] is symmetric
// positive semi-definite and solved exactly when x solves the complex one;
// conjugate gradients on it take the same iterates as complex CG.  The batch is
// stored once, stacked: U = [X; Z] (2 N_s x P), so that A = U^T U and B = U^T V
// with V = [Z; -X] (the row halves of U swapped, one negated): the Gram kernel
// forms both from the same loads of U, 4 N_s P^2 flops for the two triangles, the
// cost of the Hermitian product itself.
#include "kernels.h"

namespace nqs {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// tanh(x + iy) = (sinh 2x + i sin 2y) / (cosh 2x + cos 2y)
__device__ __forceinline__ double2 ctanh(double2 z) {
    const double d = cosh(2.0 * z.x) + cos(2.0 * z.y);
    return make_double2(sinh(2.0 * z.x) / d, sin(2.0 * z.y) / d);
}
// cosh(x + iy) = cosh x cos y + i sinh x sin y
__device__ __forceinline__ double2 ccosh(double2 z) {
    return make_double2(cosh(z.x) * cos(z.y), sinh(z.x) * sin(z.y));
}
__device__ __forceinline__ double2 cexp(double2 z) {
    const double m = exp(z.x);
    return make_double2(m * cos(z.y), m * sin(z.y));
}
// principal logarithm
__device__ __forceinline__ double2 clog(double2 z) {
    return make_double2(0.5 * log(cabs2(z)), atan2(z.y, z.x));
}

// ---------------------------------------------------------------------------
// tables: T[i][j] = tanh(2 W_ji); K[i] = (K_i(+1), K_i(-1)) (products over j in
// order, one thread per site)
// ---------------------------------------------------------------------------
__global__ void k_h_tables(int N, int M, const double2* __restrict__ p, double2* __restrict__ T,
                           double2* __restrict__ K) {
    const double2* a = p;
    const double2* W = p + N + M;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (long)N * M) {
        const int i = (int)(e / M), j = (int)(e - (long)i * M);
        const double2 w = W[(size_t)j * N + i];
        T[e] = ctanh(make_double2(2.0 * w.x, 2.0 * w.y));
    }
    if (e < N) {
        const int i = (int)e;
        double2 c = make_double2(1.0, 0.0);
        for (int j = 0; j < M; ++j) {
            const double2 w = W[(size_t)j * N + i];
            c = cmul(c, ccosh(make_double2(2.0 * w.x, 2.0 * w.y)));
        }
        const double2 ai = a[i];
        K[2 * i] = cmul(cexp(make_double2(-2.0 * ai.x, -2.0 * ai.y)), c);
        K[2 * i + 1] = cmul(cexp(make_double2(2.0 * ai.x, 2.0 * ai.y)), c);
    }
}

// ---------------------------------------------------------------------------
// tanh(theta_j(s)), theta_j = b_j + sum_i W_ji s_i, one thread per (row, j);
// and ln psi(s) = sum_i a_i s_i + sum_j ln cosh theta_j (principal logarithms,
// the branch the oracle takes), one thread per row
// ---------------------------------------------------------------------------
__global__ void k_h_theta(int N, int M, const double2* __restrict__ p, const int8_t* __restrict__ s,
                          long rows, double2* __restrict__ t, double2* __restrict__ t2,
                          long t2_stride) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * M) return;
    const long r = e / M;
    const int j = (int)(e - r * M);
    const double2* Wj = p + N + M + (size_t)j * N;
    const int8_t* sr = s + r * N;
    double2 th = p[N + j];
    for (int i = 0; i < N; ++i) {
        const double sv = (double)sr[i];
        th.x += Wj[i].x * sv;
        th.y += Wj[i].y * sv;
    }
    const double2 v = ctanh(th);
    t[e] = v;
    if (t2) t2[r * t2_stride + j] = v;
}

__global__ void k_h_log_psi(int N, int M, const double2* __restrict__ p,
                            const int8_t* __restrict__ s, long n, double2* __restrict__ out) {
    const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int8_t* sr = s + r * N;
    double2 v = make_double2(0.0, 0.0);
    for (int i = 0; i < N; ++i) {
        v.x += p[i].x * sr[i];
        v.y += p[i].y * sr[i];
    }
    for (int j = 0; j < M; ++j) {
        const double2* Wj = p + N + M + (size_t)j * N;
        double2 th = p[N + j];
        for (int i = 0; i < N; ++i) {
            th.x += Wj[i].x * sr[i];
            th.y += Wj[i].y * sr[i];
        }
        const double2 l = clog(ccosh(th));
        v.x += l.x;
        v.y += l.y;
    }
    out[r] = v;
}

// ---------------------------------------------------------------------------
// Metropolis, local rule (paper, Monte Carlo samplers): one wave per chain,
// lane l holds hidden units l, l + 64, ... (QM of them) and sites l, l + 64, ...
// of the chain.  Proposals draw the same Philox words as the real sampler:
// site = floor(x0 N / 2^32), u from x1, x2 (53 bits); the move is accepted iff
// u < |psi(s')/psi(s)|^2 = |K_i(s_i)|^2 prod_j |1 - s_i t_j T_ij|^2.  On
// acceptance t_j <- (t_j - s_i T_ij) / (1 - s_i t_j T_ij) = tanh(theta_j - 2 s_i W_ji).
// ---------------------------------------------------------------------------
constexpr int H_QM = 8;  // hidden units per lane, at most (M <= 512)

template <int QM>
__global__ __launch_bounds__(256) void k_h_sample(int N, int M, const double2* __restrict__ T,
                                                  const double2* __restrict__ K, int C, int Kp,
                                                  uint64_t seed, uint64_t prop_base,
                                                  int8_t* __restrict__ chains,
                                                  const double2* __restrict__ tch, int record,
                                                  int8_t* __restrict__ rec, long rec_stride,
                                                  uint8_t* __restrict__ acc_log, long log_stride,
                                                  long log_offset, uint32_t* acc_count) {
    extern __shared__ int8_t h_spins[];  // [4 waves][N]: each wave's chain
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (c >= C) return;
    int8_t* gs = chains + (size_t)c * N;
    int8_t* s = h_spins + (size_t)(threadIdx.x >> 6) * N;
    for (int i = lane; i < N; i += 64) s[i] = gs[i];
    __builtin_amdgcn_wave_barrier();
    double2 t[QM];
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int j = lane + 64 * q;
        t[q] = j < M ? tch[(size_t)c * M + j] : make_double2(0.0, 0.0);
    }
    uint32_t nacc = 0;
    for (int q0 = 0; q0 < Kp; q0 += 64) {
        // this lane's draw: proposal q0 + lane
        const uint64_t pidx = prop_base + (uint64_t)(q0 + lane);
        const uint4 x = philox10(make_uint4((uint32_t)pidx, (uint32_t)(pidx >> 32), (uint32_t)c,
                                            TAG_METROPOLIS), seed);
        const int my_site = (int)(((uint64_t)x.x * (uint64_t)N) >> 32);
        const double my_u = ((double)(x.y >> 5) * 67108864.0 + (double)(x.z >> 6)) *
                            (1.0 / 9007199254740992.0);
        const int nb = min(64, Kp - q0);
        for (int b = 0; b < nb; ++b) {
            const int i = __builtin_amdgcn_readlane(my_site, b);
            const double u = readlane(my_u, b);
            const double si = (double)s[i];
            const double2* Ti = T + (size_t)i * M;
            double part = 1.0;
            double2 fac[QM];
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                const int j = lane + 64 * q;
                if (j < M) {
                    const double2 tt = cmul(t[q], Ti[j]);
                    fac[q] = make_double2(1.0 - si * tt.x, -si * tt.y);
                    part *= cabs2(fac[q]);
                } else {
                    fac[q] = make_double2(1.0, 0.0);
                }
            }
            const double2 Ki = K[2 * i + (si > 0 ? 0 : 1)];
            const double ratio2 = cabs2(Ki) * wave_prod(part);
            const bool acc = u < ratio2;
            if (acc) {
#pragma unroll
                for (int q = 0; q < QM; ++q) {
                    const int j = lane + 64 * q;
                    if (j < M) {
                        const double2 num = make_double2(t[q].x - si * Ti[j].x, t[q].y - si * Ti[j].y);
                        t[q] = cdiv(num, fac[q]);
                    }
                }
                if (lane == 0) s[i] = (int8_t)(-(int)s[i]);
                ++nacc;
            }
            if (acc_log && lane == 0) acc_log[(size_t)c * log_stride + log_offset + q0 + b] = acc ? 1 : 0;
            __builtin_amdgcn_wave_barrier();  // the flipped spin is seen by the next proposal
        }
    }
    if (lane == 0 && acc_count) acc_count[c] += nacc;
    for (int i = lane; i < N; i += 64) {
        gs[i] = s[i];
        if (record) rec[(size_t)c * rec_stride + i] = s[i];
    }
}

// ---------------------------------------------------------------------------
// local energies of the TFIM (paper, local-estimator equation), one wave per
// sample, lanes over sites:
//   E(s) = J sum_<ab> s_a s_b - h sum_i K_i(s_i) prod_j (1 - s_i t_j T_ij)
// (the products over j in order; complex sums over the wave in a fixed order)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_h_eloc(int N, int M, const double2* __restrict__ T,
                                                const double2* __restrict__ K, int n_bonds,
                                                const int32_t* __restrict__ bonds, double J,
                                                double h, const int8_t* __restrict__ s,
                                                const double2* __restrict__ tact, long n,
                                                double2* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const long k = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (k >= n) return;
    const int8_t* sk = s + k * N;
    const double2* tk = tact + k * M;
    double2 off = make_double2(0.0, 0.0);
    for (int i = lane; i < N; i += 64) {
        const double si = (double)sk[i];
        const double2* Ti = T + (size_t)i * M;
        double2 r = K[2 * i + (si > 0 ? 0 : 1)];
        for (int j = 0; j < M; ++j) {
            const double2 tt = cmul(tk[j], Ti[j]);
            r = cmul(r, make_double2(1.0 - si * tt.x, -si * tt.y));
        }
        off.x += r.x;
        off.y += r.y;
    }
    double dg = 0.0;
    for (int b = lane; b < n_bonds; b += 64) dg += (double)sk[bonds[2 * b]] * sk[bonds[2 * b + 1]];
    const double dsum = wave_sum(dg);
    const double re = wave_sum(off.x), im = wave_sum(off.y);
    if (lane == 0) out[k] = make_double2(J * dsum - h * re, -h * im);
}

// ---------------------------------------------------------------------------
// energy statistics (one block): mean (complex), variance = mean |E - mean|^2,
// error = sqrt(variance / n); out[0..3] = mean re, variance, error, mean im
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_h_stats(const double2* __restrict__ E, long n,
                                                 double* __restrict__ out) {
    __shared__ double sh[3][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double a = 0.0, b = 0.0;
    for (long k = tid; k < n; k += 256) {
        a += E[k].x;
        b += E[k].y;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
        sh[0][wave] = a;
        sh[1][wave] = b;
    }
    __syncthreads();
    const double mr = ((sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3])) / (double)n;
    const double mi = ((sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3])) / (double)n;
    double v = 0.0;
    for (long k = tid; k < n; k += 256) {
        const double dr = E[k].x - mr, di = E[k].y - mi;
        v += dr * dr + di * di;
    }
    v = wave_sum(v);
    if (lane == 0) sh[2][wave] = v;
    __syncthreads();
    if (tid == 0) {
        const double var = ((sh[2][0] + sh[2][1]) + (sh[2][2] + sh[2][3])) / (double)n;
        out[0] = mr;
        out[1] = var;
        out[2] = sqrt(var / (double)n);
        out[3] = mi;
    }
}

// ---------------------------------------------------------------------------
// Jacobian O_k (packed columns: O_a_i = s_i, O_b_j = t_j, O_W_ji = t_j s_i)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 h_jac(int N, int M, const int8_t* sk, const double2* tk, long p) {
    if (p < N) return make_double2((double)sk[p], 0.0);
    if (p < N + M) return tk[p - N];
    const long q = p - N - M;
    const int j = (int)(q / N), i = (int)(q - (long)j * N);
    const double si = (double)sk[i];
    return make_double2(tk[j].x * si, tk[j].y * si);
}

// the complex Jacobian itself, O[k][p] (row-major, P columns)
__global__ __launch_bounds__(256) void k_h_jacobian(int N, int M, const int8_t* __restrict__ s,
                                                    const double2* __restrict__ t, long n, int P,
                                                    double2* __restrict__ O) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * P) return;
    const long k = e / P, p = e - k * P;
    O[e] = h_jac(N, M, s + k * N, t + k * M, p);
}

// column sums over row slices (FP64, rows in order): part[slice][p]
__global__ __launch_bounds__(256) void k_h_colsum(int N, int M, const int8_t* __restrict__ s,
                                                  const double2* __restrict__ t, long n, int P,
                                                  int slices, double2* __restrict__ part) {
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const long k0 = n * blockIdx.y / slices, k1 = n * (blockIdx.y + 1) / slices;
    double2 acc = make_double2(0.0, 0.0);
    for (long k = k0; k < k1; ++k) {
        const double2 o = h_jac(N, M, s + k * N, t + k * M, p);
        acc.x += o.x;
        acc.y += o.y;
    }
    part[(size_t)blockIdx.y * P + p] = acc;
}
__global__ void k_h_colsum_fin(const double2* __restrict__ part, int P, int slices, long n,
                               double2* __restrict__ mean) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    double2 a = make_double2(0.0, 0.0);
    for (int q = 0; q < slices; ++q) {
        a.x += part[(size_t)q * P + p].x;
        a.y += part[(size_t)q * P + p].y;
    }
    mean[p] = make_double2(a.x / (double)n, a.y / (double)n);
}

// The stacked, centred, scaled Jacobian: for sample k and column p,
// v = (O_kp - mean_p) / sqrt(n);  U[k][p] = Re v, U[n8 + k][p] = Im v with
// n8 = n rounded up to a multiple of 8; columns P .. ld - 1 and rows n .. n8 - 1,
// n8 + n .. 2 n8 - 1 are zero (the latter never written: the workspace starts
// zeroed).  Block: 256 columns x 4 rows, rows k0 + ...
__global__ __launch_bounds__(256) void k_h_jac_emb(int N, int M, const int8_t* __restrict__ s,
                                                   const double2* __restrict__ t, long n, long k0,
                                                   int P, const double2* __restrict__ mean,
                                                   long ld, double* __restrict__ U) {
    const long col = (long)blockIdx.x * 256 + threadIdx.x;  // in [0, ld)
    const double rs = 1.0 / sqrt((double)n);
    const long n8 = h_half_rows(n);
    for (int r = 0; r < 4; ++r) {
        const long k = k0 + (long)blockIdx.y * 4 + r;
        if (k >= n || col >= ld) continue;
        double re = 0.0, im = 0.0;
        if (col < P) {
            const double2 o = h_jac(N, M, s + k * N, t + k * M, col);
            re = (o.x - mean[col].x) * rs;
            im = (o.y - mean[col].y) * rs;
        }
        U[k * ld + col] = re;
        U[(n8 + k) * ld + col] = im;
    }
}

// The force f~ = dJ^H (E - mean E) / sqrt(n), embedded [Re | Im]:
//   Re f~ = X^T eR + Z^T eI,  Im f~ = X^T eI - Z^T eR,  e = (E - mean E) / sqrt(n),
// one pass over U = [X; Z] with two sums per column; slice partials over
// samples, then their sum in order (part: [slices][2P]).
__global__ __launch_bounds__(256) void k_h_force(const double* __restrict__ U, long n, long ld,
                                                 int P, const double2* __restrict__ E,
                                                 const double* __restrict__ stats, int slices,
                                                 double* __restrict__ part) {
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const long k0 = n * blockIdx.y / slices, k1 = n * (blockIdx.y + 1) / slices;
    const long n8 = h_half_rows(n);
    const double mr = stats[0], mi = stats[3], rs = 1.0 / sqrt((double)n);
    double fr = 0.0, fi = 0.0;
    for (long k = k0; k < k1; ++k) {
        const double x = U[k * ld + p], z = U[(n8 + k) * ld + p];
        const double er = (E[k].x - mr) * rs, ei = (E[k].y - mi) * rs;
        fr += x * er + z * ei;
        fi += x * ei - z * er;
    }
    part[(size_t)blockIdx.y * 2 * P + p] = fr;
    part[(size_t)blockIdx.y * 2 * P + P + p] = fi;
}
__global__ void k_h_sum_slices(const double* __restrict__ part, int P2, int slices,
                               double* __restrict__ out) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P2) return;
    double a = 0.0;
    for (int q = 0; q < slices; ++q) a += part[(size_t)q * P2 + p];
    out[p] = a;
}

// ---------------------------------------------------------------------------
// Gram matrices A = U^T U and B = U^T V on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64).  One block of 8 waves per (128 x 128 tile of the
// upper block triangle, slice of rows); wave w owns rows 32 (w / 2) .. + 31 and
// columns 64 (w % 2) .. + 63 of the tile, for A and for B, from the same loads
// of U (the B operand of B's products is V = [Z; -X], read from U with the row
// halves swapped).  The next 4 rows' operands are loaded before the current
// ones are multiplied.  Row slices spread the triangle's few hundred tiles over
// all compute units; each slice writes its tile partials [2][128][128], which
// k_h_gram_fin sums in slice order (deterministic).
// ---------------------------------------------------------------------------
constexpr int HG_TILE = 128;
constexpr int HG_ROWS = 16;                  // rows of U per LDS stage
constexpr int HG_LD = 3 * HG_TILE + 2;       // LDS row: p panel | q panel | V's q panel (+pad)

// U: [2 n8][ld], n8 = n rounded up to 8 (zero rows pad both halves), so every
// slice is whole 16-row stages and every 4-row step lies in one half: V's sign
// is uniform per step.  Per stage each thread moves 6 x 16 B from U into
// registers, at the top of the stage, while the waves multiply the previous
// stage out of LDS; the registers go to the other LDS buffer after the
// products (the barriers keep the loads where they are issued).
__global__ __launch_bounds__(512) void k_h_gram(const double* __restrict__ U, long n, long ld,
                                                int ntiles, long rows_per_slice,
                                                const int* __restrict__ tiles,
                                                double* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) double L[2][HG_ROWS * HG_LD];
    const int t = (int)(blockIdx.x % (unsigned)ntiles), ks = (int)(blockIdx.x / (unsigned)ntiles);
    const int tp = tiles[2 * t], tq = tiles[2 * t + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long n8 = h_half_rows(n), R = 2 * n8;
    const long r0 = (long)ks * rows_per_slice;
    const long r1 = r0 + rows_per_slice < R ? r0 + rows_per_slice : R;
    const int nst = r0 < r1 ? (int)((r1 - r0) / HG_ROWS) : 0;
    // this thread's 6 pieces of a stage: item = tid + 512 m -> row of the stage,
    // panel (0: p columns of U, 1: q columns of U, 2: q columns of V's row) and
    // 2 doubles; their LDS offsets
    int prow[6], ppan[6], loff[6], vsel[6];
    long pcol[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const int it = tid + 512 * m, pr = it >> 6, e = it & 63;
        prow[m] = pr / 3;
        ppan[m] = pr - 3 * prow[m];
        pcol[m] = (ppan[m] == 0 ? (long)tp : (long)tq) * HG_TILE + 2 * e;
        loff[m] = prow[m] * HG_LD + ppan[m] * HG_TILE + 2 * e;
        vsel[m] = ppan[m] == 2 ? 1 : 0;
    }
    v4d accA[2][4], accB[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            accA[a][b] = v4d{0, 0, 0, 0};
            accB[a][b] = v4d{0, 0, 0, 0};
        }
    const int pc = (wave >> 1) * 32 + lr, qc = (wave & 1) * 64 + lr;
    // U's row of piece m of stage st (V's panel: the row in the other half)
#define HG_SRC(m, st)                                                                   \
    (U + (r0 + (long)(st) * HG_ROWS + prow[m] +                                         \
          (long)vsel[m] * (r0 + (long)(st) * HG_ROWS + prow[m] < n8 ? n8 : -n8)) * ld +  \
     pcol[m])
    double2 g0, g1, g2, g3, g4, g5;
    if (nst > 0) {
        g0 = *(const double2*)HG_SRC(0, 0);
        g1 = *(const double2*)HG_SRC(1, 0);
        g2 = *(const double2*)HG_SRC(2, 0);
        g3 = *(const double2*)HG_SRC(3, 0);
        g4 = *(const double2*)HG_SRC(4, 0);
        g5 = *(const double2*)HG_SRC(5, 0);
        *(double2*)(&L[0][loff[0]]) = g0;
        *(double2*)(&L[0][loff[1]]) = g1;
        *(double2*)(&L[0][loff[2]]) = g2;
        *(double2*)(&L[0][loff[3]]) = g3;
        *(double2*)(&L[0][loff[4]]) = g4;
        *(double2*)(&L[0][loff[5]]) = g5;
    }
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const int nx = st + 1 < nst ? st + 1 : st;  // (the last stage reloads itself, unused)
        g0 = *(const double2*)HG_SRC(0, nx);
        g1 = *(const double2*)HG_SRC(1, nx);
        g2 = *(const double2*)HG_SRC(2, nx);
        g3 = *(const double2*)HG_SRC(3, nx);
        g4 = *(const double2*)HG_SRC(4, nx);
        g5 = *(const double2*)HG_SRC(5, nx);
        const double* Lb = L[st & 1];
#pragma unroll
        for (int j = 0; j < HG_ROWS / 4; ++j) {
            const long gr = r0 + (long)st * HG_ROWS + 4 * j;
            const double sg = gr < n8 ? 1.0 : -1.0;
            const double* lrow = Lb + (4 * j + lk) * HG_LD;
            double fa[2], fb[4], fv[4];
#pragma unroll
            for (int a = 0; a < 2; ++a) fa[a] = lrow[pc + a * 16];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                fb[b] = lrow[HG_TILE + qc + b * 16];
                fv[b] = sg * lrow[2 * HG_TILE + qc + b * 16];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    accA[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], accA[a][b], 0, 0, 0);
                    accB[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fv[b], accB[a][b], 0, 0, 0);
                }
        }
        double* Ln = L[(st + 1) & 1];
        *(double2*)(&Ln[loff[0]]) = g0;
        *(double2*)(&Ln[loff[1]]) = g1;
        *(double2*)(&Ln[loff[2]]) = g2;
        *(double2*)(&Ln[loff[3]]) = g3;
        *(double2*)(&Ln[loff[4]]) = g4;
        *(double2*)(&Ln[loff[5]]) = g5;
        __syncthreads();
    }
#undef HG_SRC
    double* pa_out = part + (size_t)blockIdx.x * 2 * HG_TILE * HG_TILE;
    double* pb_out = pa_out + HG_TILE * HG_TILE;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int pr = (wave >> 1) * 32 + a * 16 + acc_row<double>(lk, i);
                const int qo = (wave & 1) * 64 + b * 16 + lr;
                pa_out[pr * HG_TILE + qo] = accA[a][b][i];
                pb_out[pr * HG_TILE + qo] = accB[a][b][i];
            }
}

// Sum of the slice partials (in slice order) into A [P][ld] and B [P][ld],
// with the lower triangles mirrored (A symmetric, B antisymmetric, B's diagonal
// zero).  One block per 32 x 32 sub-block of a tile; the mirrored writes go
// through LDS so that both are coalesced.  In a diagonal tile only entries on
// or above the diagonal are taken.
__global__ __launch_bounds__(256) void k_h_gram_fin(const double* __restrict__ part, int ntiles,
                                                    int slices, const int* __restrict__ tiles,
                                                    int P, long ld, double* __restrict__ A,
                                                    double* __restrict__ B) {
    __shared__ double sa[32][33], sb[32][33];
    const int t = blockIdx.x >> 4, sub = blockIdx.x & 15;
    const int tp = tiles[2 * t], tq = tiles[2 * t + 1];
    const int i0 = (sub >> 2) * 32, j0 = (sub & 3) * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const long P0 = (long)tp * HG_TILE, Q0 = (long)tq * HG_TILE;
    const bool diag = tp == tq;
    const size_t tile_sz = 2 * HG_TILE * HG_TILE;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int ii = ty + 8 * m, jj = tx;
        const size_t e = (size_t)(i0 + ii) * HG_TILE + (j0 + jj);
        double a = 0.0, b = 0.0;
        for (int ks = 0; ks < slices; ++ks) {
            const double* pt = part + ((size_t)ks * ntiles + t) * tile_sz;
            a += pt[e];
            b += pt[HG_TILE * HG_TILE + e];
        }
        if (diag && i0 + ii == j0 + jj) b = 0.0;
        sa[ii][jj] = a;
        sb[ii][jj] = b;
        const long p = P0 + i0 + ii, q = Q0 + j0 + jj;
        if ((!diag || i0 + ii <= j0 + jj) && p < P && q < P) {
            A[p * ld + q] = a;
            B[p * ld + q] = b;
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int jj = ty + 8 * m, ii = tx;  // source element (ii, jj), written at (q, p)
        const long p = P0 + i0 + ii, q = Q0 + j0 + jj;
        if ((!diag || i0 + ii < j0 + jj) && p < P && q < P) {
            A[q * ld + p] = sa[ii][jj];
            B[q * ld + p] = -sb[ii][jj];
        }
    }
}

// (G + shift I) v for the real system [[A, -B], [B, A]], v = [v_r | v_i] (2P),
// the shift taken from the CG scalars:
// one wave per H_MV_RW rows p of A and B, each row read once for both halves of
// the output; the products' dot v.(G + shift I) v is summed per block into
// dpart (in a fixed order) for the CG step.
constexpr int H_MV_RW = 4;
int h_matvec_blocks(int P) { return (P + 4 * H_MV_RW - 1) / (4 * H_MV_RW); }

__global__ __launch_bounds__(256) void k_h_matvec(const double* __restrict__ G, int P, long ld,
                                                  const double* __restrict__ v,
                                                  double* __restrict__ out,
                                                  double* __restrict__ dpart,
                                                  const CgScalars* __restrict__ sc) {
    if (sc->done) return;
    __shared__ double sh[4];
    const double shift = sc->shift;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long p0 = ((long)blockIdx.x * 4 + wave) * H_MV_RW;
    const double* A = G;
    const double* B = G + (size_t)P * ld;
    const double* vr = v;
    const double* vi = v + P;
    double ar[H_MV_RW], ai[H_MV_RW];
#pragma unroll
    for (int r = 0; r < H_MV_RW; ++r) ar[r] = ai[r] = 0.0;
    for (long q = 4 * lane; q < P; q += 256) {
        if (q + 4 <= P) {
            const double x0 = vr[q], x1 = vr[q + 1], x2 = vr[q + 2], x3 = vr[q + 3];
            const double y0 = vi[q], y1 = vi[q + 1], y2 = vi[q + 2], y3 = vi[q + 3];
#pragma unroll
            for (int r = 0; r < H_MV_RW; ++r) {
                if (p0 + r >= P) break;
                const double* ga = A + (p0 + r) * ld + q;
                const double* gb = B + (p0 + r) * ld + q;
                const double2 a01 = *(const double2*)ga, a23 = *(const double2*)(ga + 2);
                const double2 b01 = *(const double2*)gb, b23 = *(const double2*)(gb + 2);
                ar[r] += ((a01.x * x0 - b01.x * y0) + (a01.y * x1 - b01.y * y1)) +
                         ((a23.x * x2 - b23.x * y2) + (a23.y * x3 - b23.y * y3));
                ai[r] += ((b01.x * x0 + a01.x * y0) + (b01.y * x1 + a01.y * y1)) +
                         ((b23.x * x2 + a23.x * y2) + (b23.y * x3 + a23.y * y3));
            }
        } else {  // ragged end of the row
            for (long qq = q; qq < P; ++qq)
#pragma unroll
                for (int r = 0; r < H_MV_RW; ++r)
                    if (p0 + r < P) {
                        const double a = A[(p0 + r) * ld + qq], b = B[(p0 + r) * ld + qq];
                        ar[r] += a * vr[qq] - b * vi[qq];
                        ai[r] += b * vr[qq] + a * vi[qq];
                    }
        }
    }
    double dot = 0.0;
#pragma unroll
    for (int r = 0; r < H_MV_RW; ++r) {
        const double sr = wave_sum(ar[r]), si = wave_sum(ai[r]);
        const long p = p0 + r;
        if (p < P) {
            const double orr = sr + shift * vr[p], oi = si + shift * vi[p];
            if (lane == 0) {
                out[p] = orr;
                out[P + p] = oi;
            }
            dot += orr * vr[p] + oi * vi[p];
        }
    }
    if (lane == 0) sh[wave] = dot;
    __syncthreads();
    if (threadIdx.x == 0) dpart[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// out[p] = in[p] + c x_p, x_p = x[p] + i x[P + p] (the embedding of a complex
// vector), c complex; optionally with a second vector: + c2 x2_p.
__global__ void k_h_axpy(int P, const double2* __restrict__ in, double cr, double ci,
                         const double* __restrict__ x, double c2r, double c2i,
                         const double* __restrict__ x2, double2* __restrict__ out) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const double2 v = in[p];
    const double2 xv = make_double2(x[p], x[P + p]);
    double2 r = make_double2(v.x + cr * xv.x - ci * xv.y, v.y + cr * xv.y + ci * xv.x);
    if (x2) {
        const double2 yv = make_double2(x2[p], x2[P + p]);
        r.x += c2r * yv.x - c2i * yv.y;
        r.y += c2r * yv.y + c2i * yv.x;
    }
    out[p] = r;
}

// lower triangle of the real embedding E = [[A, -B], [B, A]] of G = A + i B
__global__ void k_h_embed(const double* __restrict__ A, const double* __restrict__ B, int P,
                          long ld, double* __restrict__ E, long lde) {
    const long j = (long)blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
    if (j > i || j >= 2L * P) return;
    const long ia = i < P ? i : i - P, ja = j < P ? j : j - P;
    double v;
    if ((i < P) == (j < P)) v = A[ia * ld + ja];
    else v = B[ia * ld + ja];  // (i >= P > j: the lower-left block, + Im G)
    E[i * lde + j] = v;
}

// interleaved complex vector <-> embedding [re..., im...]
__global__ void k_h_split(int P, const double2* __restrict__ z, double* __restrict__ emb) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    emb[p] = z[p].x;
    emb[P + p] = z[p].y;
}
__global__ void k_h_join(int P, const double* __restrict__ emb, double2* __restrict__ z) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    z[p] = make_double2(emb[p], emb[P + p]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nbk(long n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_h_tables(hipStream_t st, int N, int M, const double2* p, double2* T, double2* K) {
    const long n = (long)N * M > N ? (long)N * M : N;
    k_h_tables<<<nbk(n, 256), 256, 0, st>>>(N, M, p, T, K);
}
void launch_h_theta(hipStream_t st, int N, int M, const double2* p, const int8_t* s, long rows,
                    double2* t, double2* t2, long t2_stride) {
    if (rows <= 0) return;
    k_h_theta<<<nbk(rows * M, 256), 256, 0, st>>>(N, M, p, s, rows, t, t2, t2_stride);
}
void launch_h_log_psi(hipStream_t st, int N, int M, const double2* p, const int8_t* s, long n,
                      double2* out) {
    if (n <= 0) return;
    k_h_log_psi<<<nbk(n, 128), 128, 0, st>>>(N, M, p, s, n, out);
}
int h_max_hidden() { return 64 * H_QM; }
void launch_h_sample(hipStream_t st, int N, int M, const double2* T, const double2* K,
                     const SampleArgs& a, const double2* tch) {
    const unsigned nb = nbk(a.C, 4);
    const int qm = (M + 63) / 64;
    const size_t lds = 4 * (size_t)N;
#define H_SAMPLE(Q)                                                                            \
    k_h_sample<Q><<<nb, 256, lds, st>>>(N, M, T, K, a.C, a.K, a.seed, a.prop_base, a.s, tch,   \
                                      a.record, a.rec, a.rec_stride, a.acc_log, a.log_stride, \
                                      a.log_offset, a.acc_count)
    if (qm <= 1) H_SAMPLE(1);
    else if (qm <= 2) H_SAMPLE(2);
    else if (qm <= 4) H_SAMPLE(4);
    else H_SAMPLE(8);
#undef H_SAMPLE
}
void launch_h_eloc(hipStream_t st, int N, int M, const double2* T, const double2* K,
                   const HamDev& H, const int8_t* s, const double2* tact, long n, double2* out) {
    if (n <= 0) return;
    k_h_eloc<<<nbk(n, 4), 256, 0, st>>>(N, M, T, K, H.n_bonds, H.bonds, H.J, H.h, s, tact, n, out);
}
void launch_h_stats(hipStream_t st, const double2* E, long n, double* out) {
    k_h_stats<<<1, 256, 0, st>>>(E, n, out);
}
constexpr int H_SLICES = 64;
size_t h_slice_bytes(int P) { return (size_t)H_SLICES * 2 * (size_t)P * 8; }
void launch_h_jacobian_emb(hipStream_t st, int N, int M, const int8_t* s, const double2* t,
                           long n, int P, long ld, double* Y, double2* mean, double* scratch) {
    double2* part = (double2*)scratch;  // [H_SLICES][P] complex
    k_h_colsum<<<dim3(nbk(P, 256), H_SLICES), 256, 0, st>>>(N, M, s, t, n, P, H_SLICES, part);
    k_h_colsum_fin<<<nbk(P, 256), 256, 0, st>>>(part, P, H_SLICES, n, mean);
    const long chunk = 65535L * 4;  // rows per launch (grid y limit)
    for (long k0 = 0; k0 < n; k0 += chunk) {
        const long m = n - k0 < chunk ? n - k0 : chunk;
        k_h_jac_emb<<<dim3(nbk(ld, 256), nbk(m, 4)), 256, 0, st>>>(N, M, s, t, n, k0, P, mean,
                                                                   ld, Y);
    }
}
void launch_h_jacobian(hipStream_t st, int N, int M, const int8_t* s, const double2* t, long n,
                       int P, double2* O) {
    if (n <= 0) return;
    k_h_jacobian<<<nbk(n * P, 256), 256, 0, st>>>(N, M, s, t, n, P, O);
}
void launch_h_force(hipStream_t st, const double* U, long n, long ld, int P, const double2* E,
                    const double* stats, double* f, double* scratch) {
    // (slices over samples)
    k_h_force<<<dim3(nbk(P, 256), H_SLICES), 256, 0, st>>>(U, n, ld, P, E, stats, H_SLICES,
                                                           scratch);
    k_h_sum_slices<<<nbk(2 * P, 256), 256, 0, st>>>(scratch, 2 * P, H_SLICES, f);
}
// Row slices of the Gram: enough (tile, slice) blocks to give every compute
// unit several, each slice at least 256 rows (a multiple of 4)
int h_gram_slices(int ntiles, long n) {
    int S = 1;
    while (S < 16 && (long)ntiles * S < 2048 && 2 * n / (2 * S) >= 256) S *= 2;
    return S;
}
size_t h_gram_part_bytes(int ntiles, int slices) {
    return (size_t)ntiles * slices * 2 * HG_TILE * HG_TILE * 8;
}
void launch_h_gram(hipStream_t st, const double* U, long n, long ld, int P, const int* tiles,
                   int ntiles, int slices, double* part, double* G) {
    const long R = 2 * h_half_rows(n);  // rows of U (a multiple of 16)
    long rps = (R + slices - 1) / slices;
    rps = (rps + HG_ROWS - 1) / HG_ROWS * HG_ROWS;
    k_h_gram<<<(unsigned)(ntiles * slices), 512, 0, st>>>(U, n, ld, ntiles, rps, tiles, part);
    k_h_gram_fin<<<(unsigned)(ntiles * 16), 256, 0, st>>>(part, ntiles, slices, tiles, P, ld, G,
                                                          G + (size_t)P * ld);
}
void launch_h_matvec(hipStream_t st, const double* G, int P, long ld, const double* v,
                     double* out, double* dpart, CgScalars* sc) {
    k_h_matvec<<<h_matvec_blocks(P), 256, 0, st>>>(G, P, ld, v, out, dpart, sc);
}
void launch_h_axpy(hipStream_t st, int P, const double2* in, double cr, double ci, const double* x,
                   double c2r, double c2i, const double* x2, double2* out) {
    k_h_axpy<<<nbk(P, 256), 256, 0, st>>>(P, in, cr, ci, x, c2r, c2i, x2, out);
}
void launch_h_embed(hipStream_t st, const double* G, int P, long ld, double* E, long lde) {
    k_h_embed<<<dim3(nbk(2L * P, 256), (unsigned)(2 * P)), 256, 0, st>>>(G, G + (size_t)P * ld, P,
                                                                         ld, E, lde);
}
void launch_h_split(hipStream_t st, int P, const double2* z, double* emb) {
    k_h_split<<<nbk(P, 256), 256, 0, st>>>(P, z, emb);
}
void launch_h_join(hipStream_t st, int P, const double* emb, double2* z) {
    k_h_join<<<nbk(P, 256), 256, 0, st>>>(P, emb, z);
}

}  // namespace nqs
