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
// Layout: a wave handles SB samples at once; lanes run over sites (TFIM) or
// bonds (Heisenberg) in chunks of 64, hidden units are walked sequentially
// with the sample's tanh(theta_j) as a wave-uniform (scalar) operand and
// T = tanh(2W) read from the hidden-major table (row j contiguous in sites).
#include "kernels.h"

namespace nqs {

constexpr int SB = 4;        // samples per wave
constexpr int LOGCHUNK = 64; // FP32: fold partial products into logs this often

template <typename R>
__device__ __forceinline__ double ratio_from(R prod, R logacc, R kfac) {
    if constexpr (sizeof(R) == 8) return (double)(kfac * prod);
    else return (double)__expf(kfac + logacc + __logf(prod));
}

template <typename R>
__global__ __launch_bounds__(256) void k_eloc_tfim(Dims d, const R* __restrict__ Tj,
                                                   const R* __restrict__ Ks, HamDev H,
                                                   const int8_t* __restrict__ s,
                                                   const R* __restrict__ tact, long n,
                                                   double* __restrict__ out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long k0 = ((long)blockIdx.x * 4 + wave) * SB;
    if (k0 >= n) return;
    const int N = d.N, M = d.M, Mw = d.Mw, Nw = d.Nw;
    long kr[SB];
#pragma unroll
    for (int r = 0; r < SB; ++r) kr[r] = (k0 + r < n) ? k0 + r : k0;  // duplicate, masked later
    double hsum[SB], diag[SB];
#pragma unroll
    for (int r = 0; r < SB; ++r) { hsum[r] = 0.0; diag[r] = 0.0; }

    for (int i0 = 0; i0 < N; i0 += 64) {
        const int i = i0 + lane;
        const bool valid = i < N;
        R sgn[SB], prod[SB], lacc[SB];
#pragma unroll
        for (int r = 0; r < SB; ++r) {
            sgn[r] = valid ? (R)s[kr[r] * N + i] : (R)0;
            prod[r] = (R)1;
            lacc[r] = (R)0;
        }
        for (int j0 = 0; j0 < M; j0 += LOGCHUNK) {
            const int j1 = min(M, j0 + LOGCHUNK);
            for (int j = j0; j < j1; ++j) {
                const R Tv = Tj[(size_t)j * Nw + i];
#pragma unroll
                for (int r = 0; r < SB; ++r) {
                    const R tj = tact[kr[r] * Mw + j];
                    prod[r] *= (R)1 - sgn[r] * tj * Tv;
                }
            }
            if constexpr (sizeof(R) == 4) {
#pragma unroll
                for (int r = 0; r < SB; ++r) { lacc[r] += __logf(prod[r]); prod[r] = (R)1; }
            }
        }
        if (valid) {
#pragma unroll
            for (int r = 0; r < SB; ++r) {
                const R kf = Ks[2 * i + (sgn[r] < 0)];
                hsum[r] += ratio_from<R>(prod[r], lacc[r], kf);
            }
        }
    }
    for (int b = lane; b < H.n_bonds; b += 64) {
        const int ia = H.bonds[2 * b], ib = H.bonds[2 * b + 1];
#pragma unroll
        for (int r = 0; r < SB; ++r) diag[r] += (double)(s[kr[r] * N + ia] * s[kr[r] * N + ib]);
    }
#pragma unroll
    for (int r = 0; r < SB; ++r) {
        const double e = H.J * wave_sum(diag[r]) - H.h * wave_sum(hsum[r]);
        if (lane == 0 && k0 + r < n) out[k0 + r] = e;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_eloc_heis(Dims d, const R* __restrict__ Tj,
                                                   const R* __restrict__ Ks, HamDev H,
                                                   const int8_t* __restrict__ s,
                                                   const R* __restrict__ tact, long n,
                                                   double* __restrict__ out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long k0 = ((long)blockIdx.x * 4 + wave) * SB;
    if (k0 >= n) return;
    const int N = d.N, M = d.M, Mw = d.Mw, Nw = d.Nw;
    long kr[SB];
#pragma unroll
    for (int r = 0; r < SB; ++r) kr[r] = (k0 + r < n) ? k0 + r : k0;
    double off[SB], diag[SB];
#pragma unroll
    for (int r = 0; r < SB; ++r) { off[r] = 0.0; diag[r] = 0.0; }

    for (int b0 = 0; b0 < H.n_bonds; b0 += 64) {
        const int b = b0 + lane;
        const bool valid = b < H.n_bonds;
        const int ia = valid ? H.bonds[2 * b] : 0, ib = valid ? H.bonds[2 * b + 1] : 0;
        R sa[SB], anti[SB], prod[SB], lacc[SB];
#pragma unroll
        for (int r = 0; r < SB; ++r) {
            const int xa = s[kr[r] * N + ia], xb = s[kr[r] * N + ib];
            sa[r] = (R)xa;
            anti[r] = (valid && xa != xb) ? (R)1 : (R)0;
            if (valid) diag[r] += (double)(xa * xb);
            prod[r] = (R)1;
            lacc[r] = (R)0;
        }
        for (int j0 = 0; j0 < M; j0 += LOGCHUNK) {
            const int j1 = min(M, j0 + LOGCHUNK);
            for (int j = j0; j < j1; ++j) {
                const R ta = Tj[(size_t)j * Nw + ia], tb = Tj[(size_t)j * Nw + ib];
                const R TT = (R)1 - ta * tb, Td = ta - tb;
#pragma unroll
                for (int r = 0; r < SB; ++r) {
                    const R tj = tact[kr[r] * Mw + j];
                    prod[r] *= TT - sa[r] * tj * Td;
                }
            }
            if constexpr (sizeof(R) == 4) {
#pragma unroll
                for (int r = 0; r < SB; ++r) { lacc[r] += __logf(prod[r]); prod[r] = (R)1; }
            }
        }
        if (valid) {
            double elem = 2.0 * H.J;
            if (H.sub && ((H.sub[ia] + H.sub[ib]) & 1)) elem = -elem;
#pragma unroll
            for (int r = 0; r < SB; ++r) {
                if (anti[r] != (R)0) {
                    const int xa = (int)sa[r];
                    const R kab = sizeof(R) == 8 ? Ks[2 * ia + (xa < 0)] * Ks[2 * ib + (xa > 0)]
                                                 : Ks[2 * ia + (xa < 0)] + Ks[2 * ib + (xa > 0)];
                    off[r] += elem * ratio_from<R>(prod[r], lacc[r], kab);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < SB; ++r) {
        const double e = H.J * wave_sum(diag[r]) + wave_sum(off[r]);
        if (lane == 0 && k0 + r < n) out[k0 + r] = e;
    }
}

void launch_eloc(hipStream_t st, const Dims& d, int prec, const Tables& t, const HamDev& H,
                 const int8_t* s, const void* tact, long n, double* out) {
    if (n <= 0) return;
    const int nb = (int)((n + 4 * SB - 1) / (4 * SB));
    if (prec == 0) {
        if (H.kind == 0)
            k_eloc_tfim<double><<<nb, 256, 0, st>>>(d, (const double*)t.Tj, (const double*)t.Ks, H,
                                                    s, (const double*)tact, n, out);
        else
            k_eloc_heis<double><<<nb, 256, 0, st>>>(d, (const double*)t.Tj, (const double*)t.Ks, H,
                                                    s, (const double*)tact, n, out);
    } else {
        if (H.kind == 0)
            k_eloc_tfim<float><<<nb, 256, 0, st>>>(d, (const float*)t.Tj, (const float*)t.Ks, H, s,
                                                   (const float*)tact, n, out);
        else
            k_eloc_heis<float><<<nb, 256, 0, st>>>(d, (const float*)t.Tj, (const float*)t.Ks, H, s,
                                                   (const float*)tact, n, out);
    }
}

}  // namespace nqs
