// Symmetric RBM (paper: table of models, RBMSymm; symmetric-RBM equation of the
// symmetric NQS section): alpha features over a permutation group G of sites,
//   ln psi(s) = a sum_k s_k + sum_{i < alpha, g in G} ln cosh f_g^(i)(s),
//   f_g^(i)(s) = b_i + sum_k W_i[k] s[perm_g[k]].
// The model is held as its symmetric parameters psym = [a | b (alpha) | W (alpha x N)]
// (biases as flagged) and expanded, whenever they change, into the equal plain
// RBM with M = alpha |G| hidden units: hidden unit j = i |G| + g has the weights
// W_i scattered by perm_g (W[j][perm_g[k]] = W_i[k]), the bias b_i, and every
// visible bias is a.  Its tables then drive the sampler, theta and the local
// energies unchanged, in every precision form.  Derivatives with respect to psym
// are sums over the group of the plain ones (chain rule through the expansion):
//   O_a = sum_k s_k,  O_{b_i} = sum_g t_{i|G|+g},
//   O_{W_i[k]} = sum_g t_{i|G|+g} s[perm_g[k]],   t = tanh theta.
#include "kernels.h"

namespace nqs {

// psym -> the plain RBM's packed parameters [a (N) | b (M) | W (M x N)]
__global__ void k_symm_expand(int N, int G, int alpha, int vb, int hb,
                              const int32_t* __restrict__ perms, const double* __restrict__ psym,
                              double* __restrict__ out) {
    const long M = (long)alpha * G;
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    const long ofs_b = vb ? N : 0, ofs_w = ofs_b + (hb ? M : 0);
    const double* b = psym + (vb ? 1 : 0);
    const double* W = b + (hb ? alpha : 0);
    if (e < M * N) {  // (j, k): every k of row j is hit once (perm_g is a bijection)
        const long j = e / N;
        const int k = (int)(e - j * N);
        const int i = (int)(j / G), g = (int)(j - (long)i * G);
        out[ofs_w + j * N + perms[(long)g * N + k]] = W[(long)i * N + k];
    }
    if (vb && e < N) out[e] = psym[0];
    if (hb && e < M) out[ofs_b + e] = b[e / G];
}

// the plain force (augmented layout [Ma][Na]: row j < M = (dW_j., db_j), row M =
// da) -> the symmetric one, each sum over the group in order
__global__ void k_symm_tie(int N, int G, int alpha, int vb, int hb, int Na,
                           const int32_t* __restrict__ perms, const double* __restrict__ grad,
                           double* __restrict__ out) {
    const int M = alpha * G;
    const int nb = vb ? 1 : 0, nh = hb ? alpha : 0;
    const int P = nb + nh + alpha * N;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= P) return;
    double v = 0.0;
    if (e < nb) {
        for (int k = 0; k < N; ++k) v += grad[(size_t)M * Na + k];
    } else if (e < nb + nh) {
        const int i = e - nb;
        for (int g = 0; g < G; ++g) v += grad[(size_t)(i * G + g) * Na + N];
    } else {
        const int q = e - nb - nh, i = q / N, k = q - i * N;
        for (int g = 0; g < G; ++g) v += grad[(size_t)(i * G + g) * Na + perms[(size_t)g * N + k]];
    }
    out[e] = v;
}

// O[r][p] = d ln psi(s_r) / d psym_p (FP64; columns P .. ld - 1 zero), one block
// per row: the row's spins and activations staged in LDS
template <typename T>
__global__ __launch_bounds__(256) void k_symm_jacobian(int N, int G, int alpha, int vb, int hb,
                                                       int Mw, const int32_t* __restrict__ perms,
                                                       const int8_t* __restrict__ s,
                                                       const T* __restrict__ t, long ld,
                                                       double* __restrict__ O) {
    extern __shared__ double sj[];  // [N] spins, then [alpha G] activations
    const long r = blockIdx.x;
    const int M = alpha * G;
    double* ss = sj;
    double* tt = sj + N;
    for (int k = threadIdx.x; k < N; k += 256) ss[k] = (double)s[r * N + k];
    for (int j = threadIdx.x; j < M; j += 256) tt[j] = (double)t[r * Mw + j];
    __syncthreads();
    const int nb = vb ? 1 : 0, nh = hb ? alpha : 0;
    const int P = nb + nh + alpha * N;
    for (long p = threadIdx.x; p < ld; p += 256) {
        double v = 0.0;
        if (p < nb) {
            for (int k = 0; k < N; ++k) v += ss[k];
        } else if (p < nb + nh) {
            const int i = (int)p - nb;
            for (int g = 0; g < G; ++g) v += tt[i * G + g];
        } else if (p < P) {
            const int q = (int)p - nb - nh, i = q / N, k = q - i * N;
            const double* ti = tt + i * G;
            for (int g = 0; g < G; ++g) v += ti[g] * ss[perms[(size_t)g * N + k]];
        }
        O[r * ld + p] = v;
    }
}

// ---------------------------------------------------------------------------
static inline unsigned nbk(long n, int b) { return (unsigned)((n + b - 1) / b); }

int symm_num_params(int N, int alpha, int vb, int hb) {
    return (vb ? 1 : 0) + (hb ? alpha : 0) + alpha * N;
}
void launch_symm_expand(hipStream_t st, int N, int G, int alpha, int vb, int hb,
                        const int32_t* perms, const double* psym, double* out) {
    const long M = (long)alpha * G;
    const long n = M * N > M ? M * N : M;
    k_symm_expand<<<nbk(n > N ? n : N, 256), 256, 0, st>>>(N, G, alpha, vb, hb, perms, psym, out);
}
void launch_symm_tie(hipStream_t st, int N, int G, int alpha, int vb, int hb, int Na,
                     const int32_t* perms, const double* grad, double* out) {
    k_symm_tie<<<nbk(symm_num_params(N, alpha, vb, hb), 256), 256, 0, st>>>(N, G, alpha, vb, hb,
                                                                           Na, perms, grad, out);
}
void launch_symm_jacobian(hipStream_t st, int prec, int N, int G, int alpha, int vb, int hb,
                          int Mw, const int32_t* perms, const int8_t* s, const void* t, long n,
                          long ld, double* O) {
    if (n <= 0) return;
    const size_t lds = 8 * ((size_t)N + (size_t)alpha * G);
    if (prec == 0)
        k_symm_jacobian<double><<<(unsigned)n, 256, lds, st>>>(N, G, alpha, vb, hb, Mw, perms, s,
                                                               (const double*)t, ld, O);
    else
        k_symm_jacobian<float><<<(unsigned)n, 256, lds, st>>>(N, G, alpha, vb, hb, Mw, perms, s,
                                                              (const float*)t, ld, O);
}

}  // namespace nqs
