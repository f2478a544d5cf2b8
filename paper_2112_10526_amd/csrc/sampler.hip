// Metropolis-Hastings sampling with a persistent per-chain wave (paper,
// Monte Carlo samplers section; local and exchange rules).
//
// A wave64 owns one chain, or two (32 lanes each) when the chains pair up.
// Lane l of a chain's L lanes keeps tanh(theta_j) for hidden units j = l + L q
// in registers for the whole launch, and the chain's configuration sits in
// LDS.  Random draws are made L at a time: lane l evaluates the Philox block
// of proposal p0 + l, and proposal p0 + q reads lane q's site/bond and
// uniform with v_readlane.
//
// Single flip of site i (local rule):
//   psi(s')/psi(s) = K_i(s_i) prod_j f_j,  f_j = 1 - s_i t_j T_ij,
//   T_ij = tanh(2 W_ji),  K_i(s) = exp(-2 a_i s) prod_j cosh(2 W_ji),
// from cosh(theta - x)/cosh(theta) = cosh x (1 - tanh(theta) tanh x) with
// x = 2 s_i W_ji; after acceptance t_j <- (t_j - s_i T_ij) / f_j (tanh
// subtraction formula; f_j is the denominator already computed).
// Exchange of an antiparallel pair (a, b) (s_b = -s_a):
//   psi(s'')/psi(s) = K_a(s_a) K_b(s_b) prod_j g_j,
//   g_j = 1 - T_ja T_jb - s_a t_j (T_ja - T_jb),
//   t_j <- (t_j (1 - T_ja T_jb) - s_a (T_ja - T_jb)) / g_j.
// FP64: the product is formed directly and u < r^2 is tested.  FP32: each
// lane's partial product goes through ln, the wave sums the logs, and
// ln u < 2 ln r is tested.
#include "kernels.h"

namespace nqs {

// 1/x: hardware reciprocal refined by two Newton steps (FP64), or the FP32
// hardware reciprocal.  The factors are in (0, 2), away from zero.
__device__ __forceinline__ double recip(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(fma(-x, y, 1.0), y, y);
    y = fma(fma(-x, y, 1.0), y, y);
    return y;
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Lanes of chain h of a wave: 64 / CPW consecutive lanes (CPW = 1 or 2 chains per
// wave).  With two chains per wave one cross-lane reduction and one accept/update
// sequence serve two proposals; each chain owns whole 16-lane rows, so the row
// reductions never mix the chains.
template <int CPW>
__device__ __forceinline__ int pick(int v, int q, int h) {  // chain h's lane q
    if constexpr (CPW == 1) return __builtin_amdgcn_readlane(v, q);
    else {
        const int v0 = __builtin_amdgcn_readlane(v, q), v1 = __builtin_amdgcn_readlane(v, 32 + q);
        return h ? v1 : v0;
    }
}
template <int CPW, typename T>
__device__ __forceinline__ T pick(T v, int q, int h) {
    if constexpr (CPW == 1) return readlane(v, q);
    else {
        const T v0 = readlane(v, q), v1 = readlane(v, 32 + q);
        return h ? v1 : v0;
    }
}
// sum / product over the chain's lanes (rows 4h / CPW ..), fixed order
template <int CPW, typename T>
__device__ __forceinline__ T chain_sum(T v, int h) {
    v = row16_sum(v);
    if constexpr (CPW == 1) return (readlane(v, 0) + readlane(v, 16)) + (readlane(v, 32) + readlane(v, 48));
    else {
        const T s0 = readlane(v, 0) + readlane(v, 16), s1 = readlane(v, 32) + readlane(v, 48);
        return h ? s1 : s0;
    }
}
template <int CPW, typename T>
__device__ __forceinline__ T chain_prod(T v, int h) {
    v = row16_prod(v);
    if constexpr (CPW == 1) return (readlane(v, 0) * readlane(v, 16)) * (readlane(v, 32) * readlane(v, 48));
    else {
        const T s0 = readlane(v, 0) * readlane(v, 16), s1 = readlane(v, 32) * readlane(v, 48);
        return h ? s1 : s0;
    }
}

// QMAX: hidden units per lane at one chain per wave (the row covers 64 QMAX).
template <typename R, int QMAX, int RULE, int CPW>
__global__ __launch_bounds__(256) void k_sample(Dims d, const R* __restrict__ Tt,
                                                const R* __restrict__ Ks, SampleArgs a) {
    constexpr int LPC = 64 / CPW;  // lanes per chain
    constexpr int Q = QMAX * CPW;  // hidden units per lane
    extern __shared__ int8_t lds_s[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane / LPC, hl = lane % LPC;
    const int c0 = (blockIdx.x * 4 + wave) * CPW;
    if (c0 >= a.C) return;  // uniform per wave (the launcher makes C a multiple of CPW)
    const int c = c0 + h;
    const int N = d.N, Mw = d.Mw;
    int8_t* s = lds_s + (wave * CPW + h) * round_up(N, 16);
    int8_t* sg = a.s + (size_t)c * N;
    for (int i = hl; i < N; i += LPC) s[i] = sg[i];
    __builtin_amdgcn_wave_barrier();

    const R* tc = (const R*)a.tch + (size_t)c * Mw;
    R t[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) t[q] = tc[hl + LPC * q];

    uint32_t n_acc = 0;
    for (int p0 = 0; p0 < a.K; p0 += LPC) {
        const uint64_t pidx = a.prop_base + (uint64_t)(p0 + hl);
        const uint4 x = philox10(make_uint4((uint32_t)pidx, (uint32_t)(pidx >> 32), (uint32_t)c,
                                            TAG_METROPOLIS), a.seed);
        int ia_l, ib_l = 0;
        if (RULE == 0) {
            ia_l = mulshift(x.x, N);
        } else {
            const int k = mulshift(x.x, a.n_bonds);
            ia_l = a.bonds[2 * k];
            ib_l = a.bonds[2 * k + 1];
        }
        const double u_l = unit53(x.y, x.z);
        // FP32 path compares logarithms; u = 0 gives -inf and always accepts
        const float lu_l = sizeof(R) == 8 ? 0.0f : logf((float)u_l);
        const int np = min(LPC, a.K - p0);
        // table rows and site factors of the next proposal are loaded one
        // proposal ahead
        R Ta[Q], Tb[Q];
        R ka_n[2], kb_n[2];
        {
            const int ia0 = pick<CPW>(ia_l, 0, h);
            const int ib0 = pick<CPW>(ib_l, 0, h);
#pragma unroll
            for (int qq = 0; qq < Q; ++qq) {
                Ta[qq] = Tt[(size_t)ia0 * Mw + hl + LPC * qq];
                Tb[qq] = RULE == 1 ? Tt[(size_t)ib0 * Mw + hl + LPC * qq] : (R)0;
            }
            ka_n[0] = Ks[2 * ia0];
            ka_n[1] = Ks[2 * ia0 + 1];
            kb_n[0] = RULE == 1 ? Ks[2 * ib0] : (R)0;
            kb_n[1] = RULE == 1 ? Ks[2 * ib0 + 1] : (R)0;
        }
        for (int q = 0; q < np; ++q) {
            const int ia = pick<CPW>(ia_l, q, h);
            const int sa = s[ia];
            R Tv[Q], Tw[Q];
#pragma unroll
            for (int qq = 0; qq < Q; ++qq) { Tv[qq] = Ta[qq]; Tw[qq] = Tb[qq]; }
            const R ka_c[2] = {ka_n[0], ka_n[1]};
            const R kb_c[2] = {kb_n[0], kb_n[1]};
            if (q + 1 < np) {
                const int ian = pick<CPW>(ia_l, q + 1, h);
                const int ibn = pick<CPW>(ib_l, q + 1, h);
#pragma unroll
                for (int qq = 0; qq < Q; ++qq) {
                    Ta[qq] = Tt[(size_t)ian * Mw + hl + LPC * qq];
                    if (RULE == 1) Tb[qq] = Tt[(size_t)ibn * Mw + hl + LPC * qq];
                }
                ka_n[0] = Ks[2 * ian];
                ka_n[1] = Ks[2 * ian + 1];
                if (RULE == 1) {
                    kb_n[0] = Ks[2 * ibn];
                    kb_n[1] = Ks[2 * ibn + 1];
                }
            }
            bool accept;
            if (RULE == 0) {
                R f[Q];
                R prod = (R)1;
#pragma unroll
                for (int qq = 0; qq < Q; ++qq) {
                    f[qq] = (R)1 - (R)sa * t[qq] * Tv[qq];
                    prod *= f[qq];
                }
                const R kf = sa < 0 ? ka_c[1] : ka_c[0];
                if constexpr (sizeof(R) == 8) {
                    const double r = chain_prod<CPW>(prod, h) * kf;
                    accept = pick<CPW>(u_l, q, h) < r * r;
                } else {
                    const float lr = chain_sum<CPW>(__logf(prod), h) + kf;
                    accept = pick<CPW>(lu_l, q, h) < 2.0f * lr;
                }
                if (accept) {
#pragma unroll
                    for (int qq = 0; qq < Q; ++qq) t[qq] = (t[qq] - (R)sa * Tv[qq]) * recip(f[qq]);
                    s[ia] = (int8_t)-sa;  // every lane of the chain stores the same value
                }
            } else {
                const int ib = pick<CPW>(ib_l, q, h);
                const int sb = s[ib];
                // the ratio is formed for every chain of the wave (the cross-lane
                // reduction runs outside divergent code); a bond with equal spins
                // is the identity move, accepted with ratio 1
                R g[Q], TT[Q], Td[Q];
                R prod = (R)1;
#pragma unroll
                for (int qq = 0; qq < Q; ++qq) {
                    const R ta = Tv[qq], tb = Tw[qq];
                    TT[qq] = (R)1 - ta * tb;
                    Td[qq] = (R)sa * (ta - tb);
                    g[qq] = TT[qq] - t[qq] * Td[qq];
                    prod *= g[qq];
                }
                const R ka = sa < 0 ? ka_c[1] : ka_c[0], kb = sb < 0 ? kb_c[1] : kb_c[0];
                bool take;
                if constexpr (sizeof(R) == 8) {
                    const double r = chain_prod<CPW>(prod, h) * ka * kb;
                    take = pick<CPW>(u_l, q, h) < r * r;
                } else {
                    const float lr = chain_sum<CPW>(__logf(prod), h) + ka + kb;
                    take = pick<CPW>(lu_l, q, h) < 2.0f * lr;
                }
                const bool ident = sa == sb;
                accept = ident || take;
                if (!ident && take) {
#pragma unroll
                    for (int qq = 0; qq < Q; ++qq) t[qq] = (t[qq] * TT[qq] - Td[qq]) * recip(g[qq]);
                    s[ia] = (int8_t)sb;
                    s[ib] = (int8_t)sa;
                }
            }
            n_acc += accept ? 1u : 0u;
            if (a.acc_log && hl == 0)
                a.acc_log[(size_t)c * a.log_stride + a.log_offset + p0 + q] = accept ? 1 : 0;
        }
    }
    __builtin_amdgcn_wave_barrier();
    for (int i = hl; i < N; i += LPC) {
        sg[i] = s[i];
        if (a.record) a.rec[(size_t)c * a.rec_stride + i] = s[i];
    }
    if (a.acc_count && hl == 0) a.acc_count[c] += n_acc;
}

template <typename R, int QMAX>
static void launch_q(hipStream_t st, const Dims& d, int rule, const Tables& t,
                     const SampleArgs& a) {
    // two chains per wave when the chains pair up and a lane's registers allow
    // (FP32 up to 8 x 2 hidden units per lane, FP64 up to 4 x 2)
    constexpr bool PAIR = QMAX <= (sizeof(R) == 4 ? 8 : 4);
    const int cpw = (PAIR && a.C % 2 == 0) ? 2 : 1;
    const dim3 grid((a.C + 4 * cpw - 1) / (4 * cpw));
    const size_t lds = 4 * cpw * (size_t)round_up(d.N, 16);
    if constexpr (PAIR) {
        if (cpw == 2) {
            if (rule == 0)
                k_sample<R, QMAX, 0, 2><<<grid, 256, lds, st>>>(d, (const R*)t.Tt, (const R*)t.Ks, a);
            else
                k_sample<R, QMAX, 1, 2><<<grid, 256, lds, st>>>(d, (const R*)t.Tt, (const R*)t.Ks, a);
            return;
        }
    }
    if (rule == 0)
        k_sample<R, QMAX, 0, 1><<<grid, 256, lds, st>>>(d, (const R*)t.Tt, (const R*)t.Ks, a);
    else
        k_sample<R, QMAX, 1, 1><<<grid, 256, lds, st>>>(d, (const R*)t.Tt, (const R*)t.Ks, a);
}

template <typename R>
static void launch_r(hipStream_t st, const Dims& d, int rule, const Tables& t,
                     const SampleArgs& a) {
    if (d.QM <= 1) launch_q<R, 1>(st, d, rule, t, a);
    else if (d.QM <= 2) launch_q<R, 2>(st, d, rule, t, a);
    else if (d.QM <= 4) launch_q<R, 4>(st, d, rule, t, a);
    else if (d.QM <= 8) launch_q<R, 8>(st, d, rule, t, a);
    else if (d.QM <= 16) launch_q<R, 16>(st, d, rule, t, a);
    else launch_q<R, 32>(st, d, rule, t, a);
}

// Caller guarantees d.QM <= 32 (M <= 2048).
void launch_sample(hipStream_t st, const Dims& d, int prec, int rule, const Tables& t,
                   const SampleArgs& a) {
    if (a.C <= 0 || a.K <= 0) return;
    if (prec == 0) launch_r<double>(st, d, rule, t, a);
    else launch_r<float>(st, d, rule, t, a);
}

}  // namespace nqs
