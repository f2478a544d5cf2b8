// Plain FP64 CPU oracle for the RBM variational-Monte-Carlo hot path of the
// NetKet 3 paper (arXiv 2112.10526).
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
// baseline leg of the benchmark load this library.  It shares no code, header,
// table or constant with the HIP library; it is written to be read against the
// paper, not to be fast.  Every floating-point value is double; transcendental
// functions are the C library's.
//
// Parameter vector (full layout, absent biases passed as zeros):
//   [a (N) | b (M) | W (M x N, row-major: W[j*N + i] couples hidden j, site i)]
//
// Spin configurations are int8 with values +1 / -1.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator, written from its published definition
// (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11): ten rounds of the Philox S-box on a 4-word counter, with the 2-word
// key advanced by the Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct Words4 { uint32_t w[4]; };

Words4 philox_round(const Words4& x, uint32_t k0, uint32_t k1) {
    const uint64_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    const uint64_t p0 = m0 * x.w[0];
    const uint64_t p1 = m1 * x.w[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    Words4 y;
    y.w[0] = hi1 ^ x.w[1] ^ k0;
    y.w[1] = lo1;
    y.w[2] = hi0 ^ x.w[3] ^ k1;
    y.w[3] = lo0;
    return y;
}

Words4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed) {
    Words4 x{{c0, c1, c2, c3}};
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        x = philox_round(x, k0, k1);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x;
}

// Counter of the draw for proposal p of global chain g, stream tag t:
// (p low word, p high word, g, t).  Tags: 0 Metropolis, 1 chain start.
Words4 draw(uint64_t p, uint32_t g, uint32_t tag, uint64_t seed) {
    return philox((uint32_t)p, (uint32_t)(p >> 32), g, tag, seed);
}

// Uniform index in [0, n) from one 32-bit word by multiply-shift.
int pick(uint32_t x, int n) { return (int)(((uint64_t)x * (uint64_t)n) >> 32); }

// Uniform double in [0, 1) from 27 + 26 random bits.
double uniform53(uint32_t x1, uint32_t x2) {
    return ((double)(x1 >> 5) * 67108864.0 + (double)(x2 >> 6)) * (1.0 / 9007199254740992.0);
}

// ---------------------------------------------------------------------------
// RBM log-amplitude (paper, table of models: a dense layer followed by a
// nonlinearity with alpha*N features; with log cosh as for the symmetric RBM):
//   ln psi(s) = sum_i a_i s_i + sum_j ln cosh( b_j + sum_i W_ji s_i )
// ---------------------------------------------------------------------------
struct Rbm {
    int N, M;
    const double* a;
    const double* b;
    const double* W;
};

Rbm make_rbm(int N, int M, const double* p) {
    return Rbm{N, M, p, p + N, p + N + M};
}

double theta_j(const Rbm& r, const int8_t* s, int j) {
    double th = r.b[j];
    for (int i = 0; i < r.N; ++i) th += r.W[(size_t)j * r.N + i] * s[i];
    return th;
}

double log_psi(const Rbm& r, const int8_t* s) {
    double v = 0.0;
    for (int i = 0; i < r.N; ++i) v += r.a[i] * s[i];
    for (int j = 0; j < r.M; ++j) v += std::log(std::cosh(theta_j(r, s, j)));
    return v;
}

// ---------------------------------------------------------------------------
// Hamiltonians (paper: transverse-field Ising equation; Heisenberg operator).
//   TFIM:       H = J sum_<ab> sz_a sz_b - h sum_i sx_i
//   Heisenberg: H = J sum_<ab> (sx sx + sy sy + sz sz)   (Pauli matrices)
// Heisenberg with a sublattice array: the Marshall-rotated operator
// U H U^dagger with U = prod_{i in sublattice 1} sz_i, whose off-diagonal
// element on bond (a, b) is multiplied by (-1)^(sub_a + sub_b).
// ---------------------------------------------------------------------------
struct Ham {
    int kind;           // 0 = TFIM, 1 = Heisenberg
    int n_bonds;
    const int32_t* bonds;
    double J, h;
    const int8_t* sub;  // may be null
};

double diagonal(const Ham& H, const int8_t* s) {
    double e = 0.0;
    for (int k = 0; k < H.n_bonds; ++k)
        e += H.J * s[H.bonds[2 * k]] * s[H.bonds[2 * k + 1]];
    return e;
}

// Local estimator (paper, local-estimator equation):
//   E(s) = sum_{s'} <s|H|s'> psi(s') / psi(s)
// with every ratio evaluated as exp(ln psi(s') - ln psi(s)).
double local_energy(const Rbm& r, const Ham& H, const int8_t* s) {
    const int N = r.N;
    std::vector<int8_t> sp(s, s + N);
    const double lp = log_psi(r, s);
    double e = diagonal(H, s);
    if (H.kind == 0) {
        for (int i = 0; i < N; ++i) {
            sp[i] = (int8_t)-sp[i];
            e += -H.h * std::exp(log_psi(r, sp.data()) - lp);
            sp[i] = s[i];
        }
    } else {
        for (int k = 0; k < H.n_bonds; ++k) {
            const int a = H.bonds[2 * k], b = H.bonds[2 * k + 1];
            if (s[a] == s[b]) continue;
            double elem = 2.0 * H.J;
            if (H.sub && ((H.sub[a] + H.sub[b]) & 1)) elem = -elem;
            sp[a] = s[b];
            sp[b] = s[a];
            e += elem * std::exp(log_psi(r, sp.data()) - lp);
            sp[a] = s[a];
            sp[b] = s[b];
        }
    }
    return e;
}

// ---------------------------------------------------------------------------
// Complex RBM (paper: complex parameters, holomorphic mapping theta -> psi):
// the same log-amplitude with a, b, W complex,
//   ln psi(s) = sum_i a_i s_i + sum_j ln cosh( b_j + sum_i W_ji s_i ).
// ln cosh is multivalued for complex arguments; every use below goes through
// a difference of two values inside exp() or a real part, which do not
// depend on the branch.  Parameters: the full layout [a | b | W] of complex
// numbers, each stored as (real, imaginary) doubles.
// ---------------------------------------------------------------------------
typedef std::complex<double> cplx;

struct RbmC {
    int N, M;
    const cplx* a;
    const cplx* b;
    const cplx* W;
};

RbmC make_rbm_c(int N, int M, const double* p) {
    const cplx* c = reinterpret_cast<const cplx*>(p);
    return RbmC{N, M, c, c + N, c + N + M};
}

cplx theta_jc(const RbmC& r, const int8_t* s, int j) {
    cplx th = r.b[j];
    for (int i = 0; i < r.N; ++i) th += r.W[(size_t)j * r.N + i] * (double)s[i];
    return th;
}

cplx log_psi_c(const RbmC& r, const int8_t* s) {
    cplx v = 0.0;
    for (int i = 0; i < r.N; ++i) v += r.a[i] * (double)s[i];
    for (int j = 0; j < r.M; ++j) v += std::log(std::cosh(theta_jc(r, s, j)));
    return v;
}

// Local estimator with complex amplitudes: sum_{s'} <s|H|s'> psi(s')/psi(s),
// every ratio evaluated as exp(ln psi(s') - ln psi(s)).
cplx local_energy_c(const RbmC& r, const Ham& H, const int8_t* s) {
    const int N = r.N;
    std::vector<int8_t> sp(s, s + N);
    const cplx lp = log_psi_c(r, s);
    cplx e = diagonal(H, s);
    if (H.kind == 0) {
        for (int i = 0; i < N; ++i) {
            sp[i] = (int8_t)-sp[i];
            e += -H.h * std::exp(log_psi_c(r, sp.data()) - lp);
            sp[i] = s[i];
        }
    } else {
        for (int k = 0; k < H.n_bonds; ++k) {
            const int a = H.bonds[2 * k], b = H.bonds[2 * k + 1];
            if (s[a] == s[b]) continue;
            double elem = 2.0 * H.J;
            if (H.sub && ((H.sub[a] + H.sub[b]) & 1)) elem = -elem;
            sp[a] = s[b];
            sp[b] = s[a];
            e += elem * std::exp(log_psi_c(r, sp.data()) - lp);
            sp[a] = s[a];
            sp[b] = s[b];
        }
    }
    return e;
}

}  // namespace

extern "C" {

int ora_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_philox4x32_10(const uint32_t* ctr, uint64_t seed, uint32_t* out) {
    Words4 x = philox(ctr[0], ctr[1], ctr[2], ctr[3], seed);
    for (int k = 0; k < 4; ++k) out[k] = x.w[k];
}

// Initial configurations of chains [chain_offset, chain_offset + C).
// Random start: spin i of global chain g is bit (i mod 32) of word
// (i / 32) mod 4 of the tag-1 draw with counter i / 128; s = 1 - 2*bit.
// Zero-magnetisation start (paper: Spin(1/2, total_sz=0)): N/2 up spins then
// N/2 down spins, shuffled by Fisher-Yates; swap k (k = 0 .. N-2) exchanges
// position N-1-k with a position drawn uniformly from [0, N-1-k] by the
// tag-1 draw with counter k.
void ora_init_chains(int N, int C, uint64_t seed, int chain_offset, int total_sz_zero,
                     int8_t* out) {
    for (int c = 0; c < C; ++c) {
        const uint32_t g = (uint32_t)(chain_offset + c);
        int8_t* s = out + (size_t)c * N;
        if (!total_sz_zero) {
            for (int i = 0; i < N; ++i) {
                Words4 x = draw((uint64_t)(i / 128), g, 1, seed);
                uint32_t bit = (x.w[(i / 32) % 4] >> (i % 32)) & 1u;
                s[i] = (int8_t)(1 - 2 * (int)bit);
            }
        } else {
            for (int i = 0; i < N; ++i) s[i] = (int8_t)(i < N / 2 ? 1 : -1);
            for (int k = 0; k + 1 < N; ++k) {
                const int i = N - 1 - k;
                Words4 x = draw((uint64_t)k, g, 1, seed);
                const int j = pick(x.w[0], i + 1);
                int8_t t = s[i];
                s[i] = s[j];
                s[j] = t;
            }
        }
    }
}

void ora_log_psi(int N, int M, const double* params, const int8_t* s, int64_t n, double* out) {
    const Rbm r = make_rbm(N, M, params);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) out[k] = log_psi(r, s + (size_t)k * N);
}

// Metropolis-Hastings sampling (paper, Monte Carlo samplers section).
// Each chain makes S * K proposals; proposal q of this call has global index
// p = prop_base + q.  Its tag-0 draw x gives:
//   local rule:    site i = pick(x0, N), s' = s with s_i flipped;
//   exchange rule: bond k = pick(x0, n_bonds); if the two spins differ s' is
//                  s with them swapped, otherwise s' = s (identity move);
//   u = uniform53(x1, x2).
// Both rules are symmetric, so the kernel correction vanishes and the move is
// accepted iff u < |psi(s')/psi(s)|^2.  After every K proposals the current
// configuration is recorded as a sample.
//
// mode 0 (definition): ln psi(s') is evaluated from scratch at every proposal.
// mode 1 (cached):     theta = W s + b is kept per chain, updated when a move is
//                      accepted and recomputed from s after every recorded
//                      sample; the ratio is exp(2 * [sum_i a_i (s'_i - s_i)
//                      + sum_j (ln cosh theta'_j - ln cosh theta_j)]).
// Outputs: updated chains, samples [C][S][N] (nullable), accept flags per
// proposal [C][S*K] (nullable), per-chain smallest |u - ratio^2| (nullable)
// and per-chain accepted counts (nullable).
void ora_sample(int N, int M, const double* params, int rule, int n_bonds,
                const int32_t* bonds, int C, int S, int K, uint64_t seed,
                uint64_t prop_base, int chain_offset, int mode, int8_t* chains,
                int8_t* samples, uint8_t* accept_log, double* margins, int64_t* n_acc) {
    const Rbm r = make_rbm(N, M, params);
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < C; ++c) {
        const uint32_t g = (uint32_t)(chain_offset + c);
        int8_t* s = chains + (size_t)c * N;
        std::vector<int8_t> sp(N);
        std::vector<double> theta(M), thetap(M);
        double lp = log_psi(r, s);
        if (mode == 1)
            for (int j = 0; j < M; ++j) theta[j] = theta_j(r, s, j);
        double margin = INFINITY;
        int64_t acc = 0;
        for (int q = 0; q < S * K; ++q) {
            const uint64_t p = prop_base + (uint64_t)q;
            Words4 x = draw(p, g, 0, seed);
            const double u = uniform53(x.w[1], x.w[2]);
            int f0 = -1, f1 = -1;  // flipped sites
            if (rule == 0) {
                f0 = pick(x.w[0], N);
            } else {
                const int k = pick(x.w[0], n_bonds);
                const int a = bonds[2 * k], b = bonds[2 * k + 1];
                if (s[a] != s[b]) { f0 = a; f1 = b; }
            }
            bool accept;
            if (f0 < 0) {
                accept = true;  // identity move: ratio 1
            } else {
                std::memcpy(sp.data(), s, N);
                sp[f0] = (int8_t)-sp[f0];
                if (f1 >= 0) sp[f1] = (int8_t)-sp[f1];
                double lpp = 0.0, dlog;
                if (mode == 0) {
                    lpp = log_psi(r, sp.data());
                    dlog = lpp - lp;
                } else {
                    dlog = 0.0;
                    for (int i = 0; i < N; ++i) dlog += r.a[i] * (sp[i] - s[i]);
                    for (int j = 0; j < M; ++j) {
                        double th = theta[j];
                        th += r.W[(size_t)j * N + f0] * (sp[f0] - s[f0]);
                        if (f1 >= 0) th += r.W[(size_t)j * N + f1] * (sp[f1] - s[f1]);
                        thetap[j] = th;
                        dlog += std::log(std::cosh(th)) - std::log(std::cosh(theta[j]));
                    }
                }
                const double ratio2 = std::exp(2.0 * dlog);
                const double m = std::fabs(u - ratio2);
                if (m < margin) margin = m;
                accept = u < ratio2;
                if (accept) {
                    std::memcpy(s, sp.data(), N);
                    if (mode == 0) lp = lpp;
                    else theta.swap(thetap);
                }
            }
            if (accept) ++acc;
            if (accept_log) accept_log[(size_t)c * S * K + q] = accept ? 1 : 0;
            if ((q + 1) % K == 0) {
                const int sample = (q + 1) / K - 1;
                if (samples) std::memcpy(samples + ((size_t)c * S + sample) * N, s, N);
                if (mode == 1)
                    for (int j = 0; j < M; ++j) theta[j] = theta_j(r, s, j);
                else
                    lp = log_psi(r, s);
            }
        }
        if (margins) margins[c] = margin;
        if (n_acc) n_acc[c] = acc;
    }
}

void ora_local_energy(int N, int M, const double* params, int kind, int n_bonds,
                      const int32_t* bonds, double J, double h, const int8_t* sub,
                      const int8_t* s, int64_t n, double* out) {
    const Rbm r = make_rbm(N, M, params);
    const Ham H{kind, n_bonds, bonds, J, h, sub};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < n; ++k) out[k] = local_energy(r, H, s + (size_t)k * N);
}

// Log-derivatives O_k(s) = d ln psi(s) / d p_k (paper, log-derivative
// equation), for the full layout [a | b | W]:
//   O_a_i = s_i,  O_b_j = tanh theta_j,  O_W_ji = tanh(theta_j) s_i.
void ora_jacobian(int N, int M, const double* params, const int8_t* s, int64_t n, double* O) {
    const Rbm r = make_rbm(N, M, params);
    const size_t P = (size_t)N + M + (size_t)M * N;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        const int8_t* sk = s + (size_t)k * N;
        double* o = O + (size_t)k * P;
        for (int i = 0; i < N; ++i) o[i] = sk[i];
        for (int j = 0; j < M; ++j) {
            const double t = std::tanh(theta_j(r, sk, j));
            o[N + j] = t;
            for (int i = 0; i < N; ++i) o[N + M + (size_t)j * N + i] = t * sk[i];
        }
    }
}

// ---------------------------------------------------------------------------
// Complex RBM entry points.  params: 2 (N + M + M N) doubles, the full layout
// of complex numbers as (real, imaginary) pairs; complex outputs likewise.
// ---------------------------------------------------------------------------
void ora_log_psi_c(int N, int M, const double* params, const int8_t* s, int64_t n, double* out) {
    const RbmC r = make_rbm_c(N, M, params);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        const cplx v = log_psi_c(r, s + (size_t)k * N);
        out[2 * k] = v.real();
        out[2 * k + 1] = v.imag();
    }
}

// Metropolis sampling of |psi|^2 for the complex RBM: the same proposals,
// draws and recording as ora_sample (local or exchange rule); a move is
// accepted iff u < |psi(s')/psi(s)|^2 = exp(2 Re[ln psi(s') - ln psi(s)]).
// mode 0: ln psi(s') from scratch at every proposal; mode 1: complex theta kept
// per chain, updated on acceptance and recomputed after every recorded sample.
void ora_sample_c(int N, int M, const double* params, int rule, int n_bonds,
                  const int32_t* bonds, int C, int S, int K, uint64_t seed,
                  uint64_t prop_base, int chain_offset, int mode, int8_t* chains,
                  int8_t* samples, uint8_t* accept_log, double* margins, int64_t* n_acc) {
    const RbmC r = make_rbm_c(N, M, params);
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < C; ++c) {
        const uint32_t g = (uint32_t)(chain_offset + c);
        int8_t* s = chains + (size_t)c * N;
        std::vector<int8_t> sp(N);
        std::vector<cplx> theta(M), thetap(M);
        cplx lp = log_psi_c(r, s);
        if (mode == 1)
            for (int j = 0; j < M; ++j) theta[j] = theta_jc(r, s, j);
        double margin = INFINITY;
        int64_t acc = 0;
        for (int q = 0; q < S * K; ++q) {
            const uint64_t p = prop_base + (uint64_t)q;
            Words4 x = draw(p, g, 0, seed);
            const double u = uniform53(x.w[1], x.w[2]);
            int f0 = -1, f1 = -1;
            if (rule == 0) {
                f0 = pick(x.w[0], N);
            } else {
                const int k = pick(x.w[0], n_bonds);
                const int a = bonds[2 * k], b = bonds[2 * k + 1];
                if (s[a] != s[b]) { f0 = a; f1 = b; }
            }
            bool accept;
            if (f0 < 0) {
                accept = true;
            } else {
                std::memcpy(sp.data(), s, N);
                sp[f0] = (int8_t)-sp[f0];
                if (f1 >= 0) sp[f1] = (int8_t)-sp[f1];
                cplx lpp = 0.0, dlog;
                if (mode == 0) {
                    lpp = log_psi_c(r, sp.data());
                    dlog = lpp - lp;
                } else {
                    dlog = 0.0;
                    for (int i = 0; i < N; ++i) dlog += r.a[i] * (double)(sp[i] - s[i]);
                    for (int j = 0; j < M; ++j) {
                        cplx th = theta[j];
                        th += r.W[(size_t)j * N + f0] * (double)(sp[f0] - s[f0]);
                        if (f1 >= 0) th += r.W[(size_t)j * N + f1] * (double)(sp[f1] - s[f1]);
                        thetap[j] = th;
                        dlog += std::log(std::cosh(th)) - std::log(std::cosh(theta[j]));
                    }
                }
                const double ratio2 = std::exp(2.0 * dlog.real());
                const double m = std::fabs(u - ratio2);
                if (m < margin) margin = m;
                accept = u < ratio2;
                if (accept) {
                    std::memcpy(s, sp.data(), N);
                    if (mode == 0) lp = lpp;
                    else theta.swap(thetap);
                }
            }
            if (accept) ++acc;
            if (accept_log) accept_log[(size_t)c * S * K + q] = accept ? 1 : 0;
            if ((q + 1) % K == 0) {
                const int sample = (q + 1) / K - 1;
                if (samples) std::memcpy(samples + ((size_t)c * S + sample) * N, s, N);
                if (mode == 1)
                    for (int j = 0; j < M; ++j) theta[j] = theta_jc(r, s, j);
                else
                    lp = log_psi_c(r, s);
            }
        }
        if (margins) margins[c] = margin;
        if (n_acc) n_acc[c] = acc;
    }
}

void ora_local_energy_c(int N, int M, const double* params, int kind, int n_bonds,
                        const int32_t* bonds, double J, double h, const int8_t* sub,
                        const int8_t* s, int64_t n, double* out) {
    const RbmC r = make_rbm_c(N, M, params);
    const Ham H{kind, n_bonds, bonds, J, h, sub};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < n; ++k) {
        const cplx e = local_energy_c(r, H, s + (size_t)k * N);
        out[2 * k] = e.real();
        out[2 * k + 1] = e.imag();
    }
}

// Holomorphic log-derivatives O_k(s) = d ln psi(s) / d p_k (complex):
//   O_a_i = s_i,  O_b_j = tanh theta_j,  O_W_ji = tanh(theta_j) s_i.
void ora_jacobian_c(int N, int M, const double* params, const int8_t* s, int64_t n,
                    double* O) {
    const RbmC r = make_rbm_c(N, M, params);
    const size_t P = (size_t)N + M + (size_t)M * N;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        const int8_t* sk = s + (size_t)k * N;
        cplx* o = reinterpret_cast<cplx*>(O) + (size_t)k * P;
        for (int i = 0; i < N; ++i) o[i] = (double)sk[i];
        for (int j = 0; j < M; ++j) {
            const cplx t = std::tanh(theta_jc(r, sk, j));
            o[N + j] = t;
            for (int i = 0; i < N; ++i) o[N + M + (size_t)j * N + i] = t * (double)sk[i];
        }
    }
}

}  // extern "C"
