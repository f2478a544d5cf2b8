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
// system (G + eps I) x = f are solved over the reals: with
//   Y = [[Re dJ, -Im dJ], [Im dJ, Re dJ]]   (2 N_s x 2 P)
// Y^T Y = [[Re G, -Im G], [Im G, Re G]], symmetric positive semi-definite, and
// [Re x; Im x] solves the embedded system exactly when x solves the complex
// one; conjugate gradients on it take the same iterates as complex CG.  Y is
// written once per batch; the Gram and the CG are the real dense kernels.
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

// The real embedding of the centred, scaled Jacobian: for sample k and column
// p, v = (O_kp - mean_p) / sqrt(n);
//   Y[k][p] = Re v, Y[k][P + p] = -Im v, Y[n + k][p] = Im v, Y[n + k][P + p] = Re v;
// columns 2P .. ld - 1 are zero.  Block: 256 columns x 4 rows, rows k0 + ...
__global__ __launch_bounds__(256) void k_h_jac_emb(int N, int M, const int8_t* __restrict__ s,
                                                   const double2* __restrict__ t, long n, long k0,
                                                   int P, const double2* __restrict__ mean,
                                                   long ld, double* __restrict__ Y) {
    const long col = (long)blockIdx.x * 256 + threadIdx.x;  // in [0, ld)
    const double rs = 1.0 / sqrt((double)n);
    for (int r = 0; r < 4; ++r) {
        const long k = k0 + (long)blockIdx.y * 4 + r;
        if (k >= n || col >= ld) continue;
        double top = 0.0, bot = 0.0;
        if (col < 2L * P) {
            const long p = col < P ? col : col - P;
            const double2 o = h_jac(N, M, s + k * N, t + k * M, p);
            const double vr = (o.x - mean[p].x) * rs, vi = (o.y - mean[p].y) * rs;
            if (col < P) {
                top = vr;
                bot = vi;
            } else {
                top = -vi;
                bot = vr;
            }
        }
        Y[k * ld + col] = top;
        Y[(n + k) * ld + col] = bot;
    }
}

// The force in the embedding: f[p'] = sum_r Y[r][p'] e_r, e = [Re dE; Im dE] / sqrt(n),
// dE = E - mean E (the stats' mean): slice partials over rows, then their sum
// in order (part: [slices][2P]).
__global__ __launch_bounds__(256) void k_h_force(const double* __restrict__ Y, long n, long ld,
                                                 int P2, const double2* __restrict__ E,
                                                 const double* __restrict__ stats, int slices,
                                                 double* __restrict__ part) {
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= P2) return;
    const long r0 = 2 * n * blockIdx.y / slices, r1 = 2 * n * (blockIdx.y + 1) / slices;
    const double mr = stats[0], mi = stats[3], rs = 1.0 / sqrt((double)n);
    double acc = 0.0;
    for (long r = r0; r < r1; ++r) {
        const double e = r < n ? (E[r].x - mr) * rs : (E[r - n].y - mi) * rs;
        acc += Y[r * ld + p] * e;
    }
    part[(size_t)blockIdx.y * P2 + p] = acc;
}
__global__ void k_h_sum_slices(const double* __restrict__ part, int P2, int slices,
                               double* __restrict__ out) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P2) return;
    double a = 0.0;
    for (int q = 0; q < slices; ++q) a += part[(size_t)q * P2 + p];
    out[p] = a;
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
void launch_h_force(hipStream_t st, const double* Y, long n, long ld, int P2, const double2* E,
                    const double* stats, double* f, double* scratch) {
    k_h_force<<<dim3(nbk(P2, 256), H_SLICES), 256, 0, st>>>(Y, n, ld, P2, E, stats, H_SLICES,
                                                            scratch);
    k_h_sum_slices<<<nbk(P2, 256), 256, 0, st>>>(scratch, P2, H_SLICES, f);
}
void launch_h_axpy(hipStream_t st, int P, const double2* in, double cr, double ci, const double* x,
                   double c2r, double c2i, const double* x2, double2* out) {
    k_h_axpy<<<nbk(P, 256), 256, 0, st>>>(P, in, cr, ci, x, c2r, c2i, x2, out);
}
void launch_h_split(hipStream_t st, int P, const double2* z, double* emb) {
    k_h_split<<<nbk(P, 256), 256, 0, st>>>(P, z, emb);
}
void launch_h_join(hipStream_t st, int P, const double* emb, double2* z) {
    k_h_join<<<nbk(P, 256), 256, 0, st>>>(P, emb, z);
}

}  // namespace nqs
