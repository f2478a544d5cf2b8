// Local energies (paper, local-estimator equation)
//   E(s) = sum_{s'} <s|H|s'> psi(s') / psi(s)
// with the connected configurations enumerated implicitly on the device:
//   TFIM:       diagonal J sum_b s_a s_b, and -h for each of the N single flips;
//   Heisenberg: diagonal J sum_b s_a s_b, and 2J (-1)^(l_a + l_b) (Marshall
//               labels, or +2J without them) for each antiparallel bond swap.
// The amplitude ratios use the product form of the sampler (see sampler.hip)
// with tanh(theta) of each sample taken from the activation rows written by
// the theta contraction.
//
// Layout: a block of 4 waves handles 4 SB samples; lanes run over sites (TFIM)
// or bonds (Heisenberg), up to ICH chunks of 64 per pass.  The hidden-major
// table T = tanh(2W) is staged in LDS JC hidden units at a time and shared by
// the block's samples; each sample's tanh(theta_j) is a wave-uniform operand,
// loaded for the whole chunk into the lanes (lane l: hidden unit j0 + l) and
// read out with v_readlane.
#include "kernels.h"

namespace nqs {

constexpr int SB = 8;         // samples per wave
constexpr int ICH = 2;        // site / bond chunks of 64 per pass
constexpr int LOGCHUNK = 64;  // FP32: fold partial products into logs this often

template <typename R>
__device__ __forceinline__ double ratio_from(R prod, R logacc, R kfac) {
    if constexpr (sizeof(R) == 8) return (double)(kfac * prod);
    else return (double)__expf(kfac + logacc + __logf(prod));
}

// Stage table rows [j0, j0 + jn) (all Nw columns) into LDS.
template <typename R>
__device__ __forceinline__ void stage_rows(R* __restrict__ dst, const R* __restrict__ Tj, int j0,
                                           int jn, int Nw) {
    const int total = jn * Nw;
    const R* src = Tj + (size_t)j0 * Nw;
    for (int base = 0; base < total; base += 256 * 8) {
        R v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + u * 256 + threadIdx.x;
            v[u] = e < total ? src[e] : (R)0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + u * 256 + threadIdx.x;
            if (e < total) dst[e] = v[u];
        }
    }
}

template <typename R, int KIND>
__global__ __launch_bounds__(256) void k_eloc(Dims d, const R* __restrict__ Tj,
                                              const R* __restrict__ Ks, HamDev H,
                                              const int8_t* __restrict__ s,
                                              const R* __restrict__ tact, long n,
                                              double* __restrict__ out, int JC) {
    extern __shared__ __align__(16) char lds_raw[];
    R* Ts = (R*)lds_raw;  // [JC][Nw]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long k0 = ((long)blockIdx.x * 4 + wave) * SB;
    const int N = d.N, M = d.M, Mw = d.Mw, Nw = d.Nw;
    const int n_items = KIND == 0 ? N : H.n_bonds;
    long kr[SB];
#pragma unroll
    for (int r = 0; r < SB; ++r) kr[r] = (k0 + r < n) ? k0 + r : (k0 < n ? k0 : 0);
    double acc[SB], diag[SB];
#pragma unroll
    for (int r = 0; r < SB; ++r) { acc[r] = 0.0; diag[r] = 0.0; }

    for (int g0 = 0; g0 < n_items; g0 += 64 * ICH) {
        int ia[ICH], ib[ICH];
        R sa[ICH][SB], prod[ICH][SB], lacc[ICH][SB];
#pragma unroll
        for (int c = 0; c < ICH; ++c) {
            const int it = g0 + 64 * c + lane;
            const bool valid = it < n_items;
            if (KIND == 0) {
                ia[c] = valid ? it : 0;
                ib[c] = 0;
            } else {
                ia[c] = valid ? H.bonds[2 * it] : 0;
                ib[c] = valid ? H.bonds[2 * it + 1] : 0;
            }
#pragma unroll
            for (int r = 0; r < SB; ++r) {
                const int xa = s[kr[r] * N + ia[c]];
                sa[c][r] = valid ? (R)xa : (R)0;
                if (KIND == 1 && valid) diag[r] += (double)(xa * s[kr[r] * N + ib[c]]);
                prod[c][r] = (R)1;
                lacc[c][r] = (R)0;
            }
        }
        for (int j0 = 0; j0 < M; j0 += JC) {
            const int jn = min(JC, M - j0);
            // the chunk's activations of the wave's samples, lane l holding hidden
            // unit j0 + l (JC <= 64), loaded ahead of the staging; the loop takes
            // each as a wave-uniform value with v_readlane
            R tv[SB];
#pragma unroll
            for (int r = 0; r < SB; ++r) tv[r] = tact[kr[r] * Mw + j0 + min(lane, jn - 1)];
            __syncthreads();
            stage_rows<R>(Ts, Tj, j0, jn, Nw);
            __syncthreads();
            if (k0 < n) {
                // the table entries of hidden unit jl + 1 are read while unit jl's
                // products are formed (the last unit's again at the end: the reads
                // stay unconditional)
                R na[ICH], nb[ICH];
#pragma unroll
                for (int c = 0; c < ICH; ++c) {
                    na[c] = Ts[ia[c]];
                    nb[c] = KIND == 1 ? Ts[ib[c]] : (R)0;
                }
                for (int jl = 0; jl < jn; ++jl) {
                    R tj[SB];
#pragma unroll
                    for (int r = 0; r < SB; ++r) tj[r] = readlane(tv[r], jl);
                    R ca[ICH], cb[ICH];
#pragma unroll
                    for (int c = 0; c < ICH; ++c) {
                        ca[c] = na[c];
                        cb[c] = nb[c];
                    }
                    const R* nrow = Ts + min(jl + 1, jn - 1) * Nw;
#pragma unroll
                    for (int c = 0; c < ICH; ++c) {
                        na[c] = nrow[ia[c]];
                        if (KIND == 1) nb[c] = nrow[ib[c]];
                    }
#pragma unroll
                    for (int c = 0; c < ICH; ++c) {
                        if (g0 + 64 * c >= n_items) continue;
                        if (KIND == 0) {
                            const R Tv = ca[c];
#pragma unroll
                            for (int r = 0; r < SB; ++r) prod[c][r] *= (R)1 - sa[c][r] * tj[r] * Tv;
                        } else {
                            const R ta = ca[c], tb = cb[c];
                            const R TT = (R)1 - ta * tb, Td = ta - tb;
#pragma unroll
                            for (int r = 0; r < SB; ++r) prod[c][r] *= TT - sa[c][r] * tj[r] * Td;
                        }
                    }
                    if constexpr (sizeof(R) == 4) {
                        if (((j0 + jl + 1) % LOGCHUNK) == 0) {
#pragma unroll
                            for (int c = 0; c < ICH; ++c)
#pragma unroll
                                for (int r = 0; r < SB; ++r) {
                                    lacc[c][r] += __logf(prod[c][r]);
                                    prod[c][r] = (R)1;
                                }
                        }
                    }
                }
            }
        }
        // fold the item contributions
#pragma unroll
        for (int c = 0; c < ICH; ++c) {
            const int it = g0 + 64 * c + lane;
            if (it >= n_items) continue;
            if (KIND == 0) {
#pragma unroll
                for (int r = 0; r < SB; ++r) {
                    const R kf = Ks[2 * ia[c] + (sa[c][r] < 0)];
                    acc[r] += ratio_from<R>(prod[c][r], lacc[c][r], kf);
                }
            } else {
                double elem = 2.0 * H.J;
                if (H.sub && ((H.sub[ia[c]] + H.sub[ib[c]]) & 1)) elem = -elem;
#pragma unroll
                for (int r = 0; r < SB; ++r) {
                    const int xa = (int)sa[c][r];
                    const int xb = s[kr[r] * N + ib[c]];
                    if (xa != xb) {
                        const R kab = sizeof(R) == 8 ? Ks[2 * ia[c] + (xa < 0)] * Ks[2 * ib[c] + (xb < 0)]
                                                     : Ks[2 * ia[c] + (xa < 0)] + Ks[2 * ib[c] + (xb < 0)];
                        acc[r] += elem * ratio_from<R>(prod[c][r], lacc[c][r], kab);
                    }
                }
            }
        }
    }
    if (k0 >= n) return;
    if (KIND == 0) {
        for (int b = lane; b < H.n_bonds; b += 64) {
            const int a0 = H.bonds[2 * b], b0 = H.bonds[2 * b + 1];
#pragma unroll
            for (int r = 0; r < SB; ++r) diag[r] += (double)(s[kr[r] * N + a0] * s[kr[r] * N + b0]);
        }
    }
#pragma unroll
    for (int r = 0; r < SB; ++r) {
        const double e = KIND == 0 ? H.J * wave_sum(diag[r]) - H.h * wave_sum(acc[r])
                                   : H.J * wave_sum(diag[r]) + wave_sum(acc[r]);
        if (lane == 0 && k0 + r < n) out[k0 + r] = e;
    }
}

template <typename R, int KIND>
static void launch_k(hipStream_t st, const Dims& d, const Tables& t, const HamDev& H,
                     const int8_t* s, const void* tact, long n, double* out, size_t lds_limit) {
    const size_t es = sizeof(R);
    // hidden rows of the table staged per chunk: as many as fit (down to one row,
    // for the largest lattices)
    int JC = 64;
    while (JC > 1 && (size_t)JC * d.Nw * es > lds_limit) JC /= 2;
    const size_t lds = (size_t)JC * d.Nw * es;
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_eloc<R, KIND>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int nb = (int)((n + 4 * SB - 1) / (4 * SB));
    k_eloc<R, KIND><<<nb, 256, lds, st>>>(d, (const R*)t.Tj, (const R*)t.Ks, H, s, (const R*)tact,
                                          n, out, JC);
}

void launch_eloc(hipStream_t st, const Dims& d, int prec, const Tables& t, const HamDev& H,
                 const int8_t* s, const void* tact, long n, double* out, size_t lds_limit) {
    if (n <= 0) return;
    if (prec == 0) {
        if (H.kind == 0) launch_k<double, 0>(st, d, t, H, s, tact, n, out, lds_limit);
        else launch_k<double, 1>(st, d, t, H, s, tact, n, out, lds_limit);
    } else {
        if (H.kind == 0) launch_k<float, 0>(st, d, t, H, s, tact, n, out, lds_limit);
        else launch_k<float, 1>(st, d, t, H, s, tact, n, out, lds_limit);
    }
}

}  // namespace nqs
