/*
 * nqs.h -- C ABI of libnqs: the hot path of neural-quantum-state variational
 * Monte Carlo for a real restricted Boltzmann machine (RBM) on spin-1/2
 * lattices, following the problem statement of the NetKet 3 paper
 * (arXiv 2112.10526): Hilbert space + Hamiltonian -> variational state (model
 * + Metropolis sampler) -> expectation values and gradient -> quantum
 * geometric tensor (QGT) solve -> stochastic-reconfiguration (SR) update.
 *
 * Conventions shared by every call
 *  - Every call returns an int status (nqs_status).  On failure the context
 *    records a message readable with nqs_last_error(); no exception crosses
 *    the ABI.  A failed call leaves device buffers it did not finish writing
 *    in an unspecified state, and leaves the context usable.
 *  - One context = one variational state bound to one HIP device and one HIP
 *    stream.  Kernels are launched asynchronously on that stream; calls that
 *    return host scalars (statistics, acceptance, solver info) synchronise the
 *    stream before returning.  A context may be used by one host thread at a
 *    time; different contexts are independent.
 *  - Device memory: the library never allocates device memory.  The caller
 *    allocates one workspace of nqs_workspace_bytes() bytes (e.g. a PyTorch
 *    uint8 tensor) and binds it with nqs_bind_workspace(); every internal
 *    buffer lives inside it.  Pointers documented as "device" must point to
 *    device memory on the context's device; "host" pointers to host memory.
 *    Input arrays are read during the call (host arrays are copied in) and
 *    remain owned by the caller.
 *  - Spin configurations are int8 with values +1 / -1, one row of n_sites
 *    bytes per configuration (paper, section on Hilbert spaces: spin-1/2
 *    local states in the sigma^z basis).
 *  - Parameters cross the boundary as float64 in the packed layout
 *    [a (n_sites, if visible bias) | b (n_hidden, if hidden bias) |
 *     W (n_hidden x n_sites, row-major; W[j*n_sites+i] couples hidden unit j
 *     to site i)], the contiguous parameter layout the paper uses for its
 *    dense Jacobian.  The RBM amplitude is
 *        ln psi(s) = sum_i a_i s_i + sum_j ln cosh(b_j + sum_i W_ji s_i)
 *    (paper, table of models, RBM: a dense layer followed by a nonlinearity
 *    with alpha * N features).
 */
#ifndef NQS_H
#define NQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nqs_ctx nqs_ctx;

typedef enum {
    NQS_OK = 0,
    NQS_EINVAL = 1,    /* bad argument, size or bond index */
    NQS_ENOMEM = 2,    /* workspace missing or too small */
    NQS_EDEVICE = 3,   /* HIP runtime error */
    NQS_ENUMERIC = 4,  /* non-finite parameter, energy or solver scalar */
    NQS_ENOTCONV = 5,  /* CG hit maxiter; the direction is still written */
    NQS_ESTATE = 6     /* call out of order (e.g. no Hamiltonian set yet) */
} nqs_status;

typedef enum { NQS_FP64 = 0, NQS_FP32 = 1, NQS_BF16 = 2, NQS_C128 = 3 } nqs_precision;
typedef enum { NQS_RULE_LOCAL = 0, NQS_RULE_EXCHANGE = 1 } nqs_rule;
typedef enum { NQS_QGT_ONTHEFLY = 0, NQS_QGT_JACOBIAN_DENSE = 1 } nqs_qgt;

/* Monte Carlo statistics of the local energies (paper, estimating
 * observables: sample mean with 1/N_s normalisation). */
typedef struct {
    double mean;        /* (1/N_s) sum_k E(s_k) */
    double variance;    /* (1/N_s) sum_k (E(s_k) - mean)^2 */
    double error;       /* sqrt(variance / N_s) */
    double acceptance;  /* accepted / proposed moves in the last nqs_sample */
} nqs_stats;

/* Result of one SR linear solve. */
typedef struct {
    int iterations;       /* CG iterations performed */
    int converged;        /* 1 if ||r|| <= tol * ||f|| */
    double rel_residual;  /* ||r|| / ||f|| from the CG recurrence */
} nqs_sr_info;

/* Settings of one fused VMC step. */
typedef struct {
    nqs_qgt qgt;        /* QGT representation for the SR solve */
    double diag_shift;  /* epsilon in (S + epsilon I) delta = f */
    double lr;          /* eta in p <- p - eta delta */
    double cg_tol;      /* relative residual tolerance */
    int cg_maxiter;     /* <= 0: min(P, 10000) */
} nqs_step_cfg;

/* What one VMC step reports back to the host. */
typedef struct {
    nqs_stats energy;
    nqs_sr_info sr;
    int status;         /* status of this context's step (batched calls) */
} nqs_step_report;

/* Runge-Kutta schemes of the TDVP step. */
typedef enum { NQS_RK_EULER = 0, NQS_RK_HEUN = 1 } nqs_rk_scheme;

/* Settings of one TDVP step (complex-parameter models only). */
typedef struct {
    nqs_rk_scheme scheme;
    double dt;              /* time step */
    double gamma_re;        /* gamma in G theta_dot = gamma f: -i for real time */
    double gamma_im;        /*   (gamma_re 0, gamma_im -1), -1 for imaginary time */
    double diag_shift;      /* epsilon added to G's diagonal */
    double cg_tol;          /* relative residual tolerance of each solve */
    int cg_maxiter;         /* <= 0: min(2 P, 10000) */
} nqs_tdvp_cfg;

/* What one TDVP step reports: one entry per evaluation of the equation of
 * motion (1 for Euler, 2 for Heun). */
typedef struct {
    int stages;
    nqs_stats energy[2];    /* energy[l].mean: real part of the mean local energy */
    double energy_im[2];    /* imaginary part of that mean */
    nqs_sr_info solve[2];
    int status;
} nqs_tdvp_report;

/* ------------------------------------------------------------------------- */
/* Context lifetime                                                          */
/* ------------------------------------------------------------------------- */

/* Create a context on HIP device `device` that launches on `hip_stream` (a
 * hipStream_t; NULL = the device's null stream).  *out receives the handle,
 * owned by the caller until nqs_destroy().  Errors: NQS_EINVAL (out NULL or
 * bad device), NQS_EDEVICE. */
int nqs_create(nqs_ctx** out, int device, void* hip_stream);

/* Release the context (the workspace stays owned by the caller). */
void nqs_destroy(nqs_ctx* ctx);

/* Message of the last failed call on this context ("" if none); owned by the
 * context, valid until the next call on it.  ctx NULL gives a static text. */
const char* nqs_last_error(const nqs_ctx* ctx);

/* Rebind the context to another stream (hipStream_t) of the same device. */
int nqs_set_stream(nqs_ctx* ctx, void* hip_stream);

/* ------------------------------------------------------------------------- */
/* Problem definition                                                         */
/* ------------------------------------------------------------------------- */

/* Transverse-field Ising model (paper, transverse-field Ising equation):
 *     H = J sum_<ab> sz_a sz_b - h sum_i sx_i .
 * bonds: host int32 [n_bonds][2], site pairs, each bond listed once (the
 * array is copied in).  Errors: NQS_EINVAL for n_sites < 2, n_bonds < 1 or a
 * site index outside [0, n_sites) or a bond joining a site to itself. */
int nqs_set_tfim(nqs_ctx* ctx, int n_sites, int n_bonds, const int32_t* bonds,
                 double J, double h);

/* Heisenberg model with Pauli matrices (paper, Heisenberg operator):
 *     H = J sum_<ab> (sx_a sx_b + sy_a sy_b + sz_a sz_b) .
 * sublattice: host int8 [n_sites] of 0/1 labels or NULL.  When given, the
 * Marshall-rotated operator U H U^dagger, U = prod over label-1 sites of
 * sz, is used: its off-diagonal element on bond (a, b) is 2J (-1)^(l_a+l_b),
 * so on a bipartite lattice it is sign-free and a real RBM can represent its
 * ground state.  Same errors as nqs_set_tfim. */
int nqs_set_heisenberg(nqs_ctx* ctx, int n_sites, int n_bonds, const int32_t* bonds,
                       double J, const int8_t* sublattice);

/* RBM ansatz with n_hidden = alpha * n_sites hidden units (paper, table of
 * models).  visible_bias / hidden_bias switch a and b on or off.  prec
 * selects the arithmetic:
 *  - NQS_FP64: FP64 everywhere (theta and the QGT contractions on the FP64
 *    matrix cores).
 *  - NQS_FP32: theta on the FP32 matrix cores; FP32 sampler and local
 *    energies; the on-the-fly QGT contractions and the force take each FP32
 *    operand as the sum of two BF16 terms on the BF16 matrix cores with FP32
 *    accumulation (about 2^-17 relative error per product; on the same sample
 *    batch CG on this operator takes 13-19 % more iterations than the FP64
 *    path); energy means, variances and every CG inner product and scalar in
 *    FP64.
 *  - NQS_BF16: as NQS_FP32, except that the W s + b contraction runs on the
 *    BF16 matrix cores with FP32 accumulation (W split into two BF16 terms).
 *  - NQS_C128: complex parameters a, b, W with the holomorphic mapping
 *    theta -> psi (paper, complex parameters; complex co-gradient and SR
 *    equations; TDVP), complex FP64 throughout.  Parameter, gradient and
 *    direction vectors hold 2 P doubles, (real, imaginary) pairs in the
 *    packed order; local energies and ln psi are (real, imaginary) pairs.
 *    The QGT is the dense holomorphic one, G = dJ^H dJ (dense Jacobian form
 *    only), solved as the equivalent real symmetric system of size 2 P on
 *    the FP64 matrix cores.  Supported with the TFIM, the local rule, both
 *    biases and n_hidden <= 512; nqs_log_psi_vjp, the batched and
 *    asynchronous steps and nqs_local_energy_noalloc reject it.
 * Requires a Hamiltonian.  Errors: NQS_EINVAL (n_hidden < 1, bad prec, or a
 * combination NQS_C128 does not support), NQS_ESTATE. */
int nqs_set_rbm(nqs_ctx* ctx, int n_hidden, int visible_bias, int hidden_bias,
                nqs_precision prec);

/* How the dense QGT system (S + eps I) x = f is solved (paper: solving linear
 * systems in the QGT section; the dense-solver and CG rows of the jVMC
 * comparison): conjugate gradients (default), or a direct solve by an in-place
 * blocked Cholesky factorisation of the FP64 S + eps I (the Gram matrix is
 * overwritten), reporting 0 iterations and a zero residual.  The Cholesky solve
 * needs S + eps I positive definite (eps > 0 unless S is), else the SR call
 * returns NQS_ENUMERIC; it takes the FP64 dense QGT (NQS_FP64 plain models,
 * symmetric models, complex models through the real embedding of G, 2P <=
 * 32768, which adds a [2P][2P] FP64 buffer to the workspace; every model adds the
 * inverses of the 32 x 32 diagonal blocks).  Set it before
 * nqs_bind_workspace (the workspace changes with it; changing it unbinds).
 * nqs_batch_step and nqs_step_begin do not take it (NQS_EINVAL). */
typedef enum { NQS_SOLVER_CG = 0, NQS_SOLVER_CHOLESKY = 1 } nqs_dense_solver;
int nqs_set_dense_solver(nqs_ctx* ctx, nqs_dense_solver solver);

/* Symmetric RBM (paper: table of models, RBMSymm; symmetric NQS section,
 * symmetric-RBM equation): alpha features over a group G of site permutations,
 *   ln psi(s) = a sum_k s_k + sum_{i < alpha, g} ln cosh(b_i + sum_k W_i[k] s[perm_g[k]]).
 * perms: host int32 [n_perms][n_sites], copied; row g is perm_g, row 0 must be
 * the identity and the rows must form a group (closed under composition).
 * Parameters (nqs_set_params / nqs_get_params, nqs_num_params of them), packed
 * [a (1, if visible_bias) | b (alpha, if hidden_bias) | W (alpha x n_sites,
 * row-major)]; gradients, SR directions and Jacobian columns use the same order.
 * The model runs as the equal plain RBM with alpha * n_perms hidden units
 * (sampler, local energies and ln psi as for nqs_set_rbm, in the chosen
 * precision: NQS_FP64, NQS_FP32 or NQS_BF16); its Jacobian (nqs_jacobian, FP64
 * [n][P] whatever the precision), force and dense QGT are over the symmetric
 * parameters (sums over G of the plain ones).  Sets the dense QGT
 * (NQS_QGT_JACOBIAN_DENSE; the SR solve takes at most 65535 samples).
 * nqs_log_psi_vjp, nqs_batch_step and nqs_step_begin return NQS_EINVAL for it.
 * Errors: NQS_EINVAL (not a group, alpha * n_perms > 2048, NQS_C128),
 * NQS_ESTATE (no Hamiltonian yet). */
int nqs_set_rbm_symm(nqs_ctx* ctx, int n_perms, const int32_t* perms, int alpha,
                     int visible_bias, int hidden_bias, nqs_precision prec);

/* Number P of packed parameters. 0 before nqs_set_rbm. */
size_t nqs_num_params(const nqs_ctx* ctx);

/* Metropolis sampler (paper, Monte Carlo samplers section).
 * rule NQS_RULE_LOCAL flips one site per proposal (MetropolisLocal);
 * NQS_RULE_EXCHANGE swaps the two spins of one bond of the Hamiltonian's
 * bond list (MetropolisExchange, conserves magnetisation).  n_chains chains
 * each record samples_per_chain samples per nqs_sample(), one every
 * sweep_size proposals; chains persist across calls.  Random numbers come
 * from Philox4x32-10 keyed by `seed`; the draw for proposal p of chain c has
 * counter (p lo, p hi, c, 0); chain starts use counter tag 1.
 * total_sz_zero starts every chain in the zero-magnetisation sector
 * (required for the exchange rule on a Heisenberg model).
 * Errors: NQS_EINVAL, NQS_ESTATE (no model). */
int nqs_set_sampler(nqs_ctx* ctx, nqs_rule rule, int n_chains, int samples_per_chain,
                    int sweep_size, uint64_t seed, int total_sz_zero);

/* Choose the QGT representation whose buffers the workspace must hold:
 * NQS_QGT_ONTHEFLY (default; no Jacobian stored) or NQS_QGT_JACOBIAN_DENSE
 * (stores the centred Jacobian [N_s][P] and the dense matrix [P][P], both in
 * FP32 for NQS_FP32/NQS_BF16 and FP64 for NQS_FP64; paper, QGT
 * implementation differences).  The dense matrix is formed on the FP64 or FP32
 * matrix cores, and for NQS_BF16 on the BF16 matrix cores from a two-term
 * BF16 split of each FP32 entry (three products, FP32 accumulation).  Must
 * precede nqs_workspace_bytes(). */
int nqs_set_qgt(nqs_ctx* ctx, nqs_qgt kind);

/* Bytes of device workspace the current configuration needs (0 if the
 * configuration is incomplete).  This is the context's HBM footprint. */
size_t nqs_workspace_bytes(const nqs_ctx* ctx);

/* Bind caller-owned device memory (>= nqs_workspace_bytes, 256-byte aligned)
 * and initialise tables and chains.  The memory must stay valid until the
 * context is destroyed or rebound.  Errors: NQS_ENOMEM (too small or NULL),
 * NQS_EINVAL (misaligned), NQS_ESTATE (incomplete configuration). */
int nqs_bind_workspace(nqs_ctx* ctx, void* dev_ptr, size_t bytes);

/* ------------------------------------------------------------------------- */
/* Parameters, chains and checkpoints                                        */
/* ------------------------------------------------------------------------- */

/* Copy P float64 parameters in (host or device pointer) and rebuild the
 * derived tables.  Errors: NQS_ENUMERIC if any value is not finite. */
int nqs_set_params(nqs_ctx* ctx, const double* p, int on_device);
int nqs_get_params(nqs_ctx* ctx, double* p, int on_device);

/* Restart every chain from its Philox start configuration and reset the
 * proposal counter to 0. */
int nqs_reset_chains(nqs_ctx* ctx);

/* Current chain configurations, int8 [n_chains][n_sites] (host or device). */
int nqs_get_chains(nqs_ctx* ctx, int8_t* out, int on_device);
int nqs_set_chains(nqs_ctx* ctx, const int8_t* in, int on_device);

/* Number of proposals every chain has made since its start. */
uint64_t nqs_proposal_count(const nqs_ctx* ctx);

/* Checkpoint blob (host memory): parameters, chains and proposal counter.
 * With blob NULL, *bytes receives the size.  nqs_set_state restores it
 * exactly, so a resumed run continues bit-for-bit. */
int nqs_get_state(nqs_ctx* ctx, void* blob, size_t* bytes);
int nqs_set_state(nqs_ctx* ctx, const void* blob, size_t bytes);

/* ------------------------------------------------------------------------- */
/* The hot path                                                              */
/* ------------------------------------------------------------------------- */

/* Metropolis-Hastings sampling (paper, Monte Carlo samplers section): every
 * chain makes n_discard_segments * sweep_size proposals that are not
 * recorded, then samples_per_chain * sweep_size proposals, recording its
 * configuration after every sweep_size of them.  A proposal s -> s' is
 * accepted iff u < |psi(s')/psi(s)|^2 with u uniform in [0,1) (53 bits from
 * the draw's words 1 and 2); the site (local rule) or bond (exchange rule)
 * is floor(word0 * n / 2^32).  The amplitude ratio uses the hidden
 * pre-activations theta = W s + b, updated per accepted move and recomputed
 * from s after every recorded sample.
 * samples_out: device int8 [n_chains][samples_per_chain][n_sites] or NULL
 * (the context keeps its own copy for nqs_expect_and_grad either way).
 * accept_log: device uint8 [n_chains][samples_per_chain*sweep_size] (1 =
 * accepted) or NULL; discarded proposals are not logged.
 * acceptance: host, receives the accepted fraction of the recorded
 * proposals, or NULL (then the call does not synchronise). */
int nqs_sample(nqs_ctx* ctx, int n_discard_segments, int8_t* samples_out,
               uint8_t* accept_log, double* acceptance);

/* Advance every chain by n_segments * sweep_size proposals without recording
 * samples (thermalisation; the same draws nqs_sample would have made). */
int nqs_thermalize(nqs_ctx* ctx, int n_segments);

/* Replace the context's current sample batch by n_samples configurations
 * (device int8 [n_samples][n_sites]; n_samples must equal n_chains *
 * samples_per_chain), so that estimators and the SR solve can be run on an
 * identical batch. */
int nqs_load_samples(nqs_ctx* ctx, const int8_t* samples, int64_t n_samples);

/* Local energies (paper, local-estimator equation):
 *     E(s) = sum_{s'} <s|H|s'> psi(s') / psi(s),
 * with the connected s' enumerated on the device (all single flips for the
 * TFIM, all antiparallel bonds for Heisenberg).  s: device int8 [n][n_sites];
 * eloc_out: device float64 [n].  Any n >= 0. */
int nqs_local_energy(nqs_ctx* ctx, const int8_t* s, int64_t n, double* eloc_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * local energies as nqs_local_energy, bit for bit, computed without the
 * context's workspace staging.  The batch's hidden activations go to a
 * static scratch array of 64 MiB that every GPU the library runs on holds
 * from module load until the process ends; the call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).  Needs
 * n * Mw * (8 for NQS_FP64, 4 otherwise) <= 64 MiB, where Mw, the padded
 * hidden width, is the larger of n_hidden + 1 rounded up to a multiple of
 * 16 and 64 * q, q the smallest power of two >= ceil(n_hidden / 64) (256
 * for 200 hidden units, so 16,384 samples of that model fit in FP64);
 * larger batches are rejected with NQS_EINVAL (split them).  All calls on one GPU
 * share its scratch, which keeps the last call's contents (nothing in it
 * needs to start at zero): calls that overlap on one GPU, from different
 * streams or contexts, race.  s: device int8 [n][n_sites]; eloc_out:
 * device float64 [n]; n >= 0. */
int nqs_local_energy_noalloc(nqs_ctx* ctx, const int8_t* s, int64_t n, double* eloc_out);

/* ln psi(s) for n configurations.  out: device, float64 [n] for NQS_FP64,
 * float32 [n] otherwise. */
int nqs_log_psi(nqs_ctx* ctx, const int8_t* s, int64_t n, void* out);

/* Vector-Jacobian product of ln psi (paper, appendix on Jacobians and their
 * products): grad_out[k] = sum_n g[n] O_k(s_n), O_k = d ln psi / d p_k.
 * g: device [n], grad_out: device [P]; both float64 for NQS_FP64 and float32
 * otherwise.  Backs the backward pass of the autograd function. */
int nqs_log_psi_vjp(nqs_ctx* ctx, const int8_t* s, int64_t n, const void* g, void* grad_out);

/* Jacobian O[n][P] = d ln psi(s_n) / d p (paper, log-derivative equation),
 * O_a = s, O_b = tanh theta, O_W[j][i] = tanh(theta_j) s_i; with center != 0
 * the column means over the n rows are subtracted and the result is scaled
 * by 1/sqrt(n) (the stored form of the dense Jacobian QGT).  O_out: device,
 * float64 for NQS_FP64 and float32 otherwise, row-major. */
int nqs_jacobian(nqs_ctx* ctx, const int8_t* s, int64_t n, void* O_out, int center);

/* Energy statistics and gradient on the current sample batch (paper,
 * force-vector equation and real-parameter gradient): local energies,
 * mean/variance/error, and grad = 2 Re Cov[O, E] = (2/N_s) O^T (E - mean).
 * E: host, or NULL.  grad: device float64 [P], or NULL.  Synchronises when E
 * is given.  Errors: NQS_ENUMERIC if the mean is not finite. */
int nqs_expect_and_grad(nqs_ctx* ctx, nqs_stats* E, double* grad);

/* Stochastic reconfiguration (paper, SR preconditioner and QGT solve):
 * solve (Re G + diag_shift I) delta = f with f the gradient of the last
 * nqs_expect_and_grad and G = (1/N_s) dO^T dO the QGT estimator on the same
 * batch, by conjugate gradients from delta = 0 with FP64 inner products,
 * stopping when ||r|| <= tol ||f|| or after maxiter iterations (<= 0 means
 * min(P, 10000)); then update p <- p - lr * delta.  kind picks the on-the-fly
 * product G v = (1/N_s) O^T (O v - mean(O v)) (no Jacobian stored) or the
 * dense matrix built once on MFMA.  delta_out: device float64 [P] or NULL.
 * info: host or NULL.  Errors: NQS_ENOTCONV (the update is still applied),
 * NQS_ENUMERIC, NQS_ESTATE (no gradient yet). */
int nqs_sr_update(nqs_ctx* ctx, nqs_qgt kind, double diag_shift, double lr, double tol,
                  int maxiter, double* delta_out, nqs_sr_info* info);

/* One VMC step: nqs_sample -> nqs_expect_and_grad -> nqs_sr_update (paper,
 * ground-state search with the SR preconditioner).  rep: host, required. */
int nqs_vmc_step(nqs_ctx* ctx, const nqs_step_cfg* cfg, nqs_step_report* rep);

/* One step of time-dependent variational Monte Carlo for a complex (NQS_C128)
 * model (paper, time propagation: the TDVP equation of motion
 * G theta_dot = gamma f and the Runge-Kutta step).  Each evaluation of the
 * equation of motion samples the current parameters (nqs_sample semantics,
 * the chains continue), forms the local energies, the force f and the dense
 * holomorphic QGT, and solves (G + diag_shift I) x = f by CG from x = 0;
 * theta_dot = gamma x.  Euler: theta <- theta + dt k1.  Heun: k1 at theta,
 * k2 at theta + dt k1, theta <- theta + dt (k1 + k2) / 2.  gamma = -i gives
 * real-time evolution, -1 imaginary time.  rep: host, required.  Errors:
 * NQS_EINVAL (not a complex model, bad settings), NQS_ENOTCONV (a solve hit
 * maxiter; the step is still taken), NQS_ENUMERIC. */
int nqs_tdvp_step(nqs_ctx* ctx, const nqs_tdvp_cfg* cfg, nqs_tdvp_report* rep);

/* One VMC step for each of n contexts (each on its own stream), issued in
 * lock-step so that the contexts' kernels overlap on the device.  Each
 * context's result is identical to an nqs_vmc_step on it alone.  cfgs and
 * reps: host arrays of n.  Returns the first non-OK status; every report's
 * `status` holds its own. */
int nqs_batch_step(nqs_ctx* const* ctxs, int n, const nqs_step_cfg* cfgs,
                   nqs_step_report* reps);

/* Asynchronous steps, for a server that advances many contexts without a
 * common barrier (each run's next step starts as soon as its previous one has
 * finished).  nqs_step_begin issues the step's sampling, local energies,
 * gradient, CG set-up and first batch of CG iterations on the context's stream
 * and returns at once; nqs_step_poll then advances every context of `ctxs`
 * that has a step in flight: further CG batches as their stop flags come back,
 * then the update and the read-back of the step's scalars.  A context whose
 * step has completed (or failed) gets completed[k] = 1 and its report in
 * reps[k] (status inside); the others get completed[k] = 0 and reps[k] is left
 * alone.  wait = 0: return after one pass over the contexts; wait = 1: return
 * once at least one step has completed or none is in flight.  Each context's
 * result is identical to an nqs_vmc_step on it alone (same kernels, same
 * fixed-order reductions).  While a step is in flight, make no other call on
 * that context except nqs_step_poll and nqs_destroy.  ctxs, reps, completed:
 * host arrays of n.  Errors: NQS_ESTATE (nqs_step_begin with a step already in
 * flight), those of nqs_vmc_step; nqs_step_poll returns the first failing
 * step's status. */
int nqs_step_begin(nqs_ctx* ctx, const nqs_step_cfg* cfg);
int nqs_step_poll(nqs_ctx* const* ctxs, int n, int wait, nqs_step_report* reps,
                  int32_t* completed);

/* ------------------------------------------------------------------------- */
/* Diagnostics                                                               */
/* ------------------------------------------------------------------------- */

/* Kernel classes timed by the event profiler. */
enum {
    NQS_PROF_SAMPLE = 0,    /* Metropolis sampler */
    NQS_PROF_THETA = 1,     /* theta contraction + tanh */
    NQS_PROF_ELOC = 2,      /* local energies */
    NQS_PROF_STATS = 3,     /* energy statistics and centring */
    NQS_PROF_QGT_W = 4,     /* w = J v (contraction 1) */
    NQS_PROF_OUTER = 5,     /* J^T z (contraction 2, force and QGT product) */
    NQS_PROF_REDUCE = 6,    /* chunk reduction + diagonal shift + CG update of x and r */
    NQS_PROF_CGVEC = 7,     /* CG direction and dot products */
    NQS_PROF_JACOBIAN = 8,  /* dense Jacobian build and centring */
    NQS_PROF_GRAM = 9,      /* dense QGT Gram matrix */
    NQS_PROF_DENSE_MV = 10, /* dense QGT product */
    NQS_PROF_UPDATE = 11,   /* parameter update and table rebuild */
    NQS_PROF_PREPARE = 12,  /* per-step layout of the batch for the contractions */
    NQS_PROF_CLASSES = 13
};

/* Time every launch of the kernel classes selected by `class_mask` (bit k =
 * class k) with HIP events on the context's stream; 0 switches timing off.
 * Enabling clears earlier totals.  Up to 16384 launches are timed; later ones
 * are neither timed nor counted.  While a CG kernel class is timed, CG
 * iterations are launched one kernel at a time (no graph replay). */
int nqs_profile_enable(nqs_ctx* ctx, uint32_t class_mask);

/* Totals since nqs_profile_enable: ms[k] summed kernel time and launches[k]
 * timed launches for k < n (n <= NQS_PROF_CLASSES); host arrays.
 * Synchronises the stream. */
int nqs_profile_read(nqs_ctx* ctx, double* ms, int64_t* launches, int n);

/* Throughput probes: the rate one instruction kind reaches on this device when
 * every lane of 8 waves per SIMD issues independent chains of it (the ceiling
 * the kernels are measured against; the datasheet's FP32 figure counts packed
 * FP32, which this library does not use).  per_second: flops per second
 * (FMA: 2 per instruction and lane; MFMA: 2 M N K per instruction), or
 * exponentials per second for NQS_PROBE_FP32_EXP.  Runs on the context's
 * device and stream (a context need not be configured), one warm-up launch
 * then three timed ones; its throwaway results go to the library's static
 * scratch (as nqs_local_energy_noalloc: calls overlapping on one GPU race). */
typedef enum {
    NQS_PROBE_FP32_FMA = 0,
    NQS_PROBE_FP64_FMA = 1,
    NQS_PROBE_FP32_EXP = 2,
    NQS_PROBE_FP64_MFMA = 3, /* v_mfma_f64_16x16x4f64 */
    NQS_PROBE_BF16_MFMA = 4  /* v_mfma_f32_16x16x32_bf16 */
} nqs_probe;
int nqs_probe_rate(nqs_ctx* ctx, nqs_probe kind, double* per_second);

/* On-the-fly CG (section "Solving linear systems"): with enable != 0 (the
 * default) a full batch of iterations is captured once as a HIP graph and
 * replayed, which removes most of the per-kernel launch cost; with 0 every
 * kernel is launched on the stream.  The results are identical either way.
 * Drops a captured graph; synchronises the stream. */
int nqs_set_cg_graphs(nqs_ctx* ctx, int enable);

/* Grouped CG iterations in nqs_batch_step (section "Solving linear systems",
 * on-the-fly QGT): with enable != 0 (the default) the on-the-fly CG of the
 * small NQS_FP32 and NQS_BF16 contexts of one batched step that share a device
 * (at least two of them; up to 32 per group, on a stream of the library's
 * own) runs as one launch per kernel class and iteration for all of them,
 * each run's blocks found through a device table of the runs' operands; with
 * 0 this context runs its own launches (as with nqs_vmc_step).  Small: samples
 * x round_up(n_hidden + 1, 16) x round_up(round_up(n_sites + 1, 16), 128) at
 * most 2^28, where launch overhead dominates a run's own launches; larger
 * contexts always run their own, side by side with the group.  Each run keeps
 * its own blocks and fixed-order sums, so its results are identical either
 * way.  Runs of one group advance in lock-step; a run that has stopped leaves
 * the group's launches from the next batch of iterations on.  Contexts whose
 * CG kernel classes are being timed (nqs_profile_enable) run their own
 * launches.  The tables sit in a static device array (no device allocation;
 * up to 8 groups, 256 runs, per device and call; further runs take their own
 * launches); the library keeps their pinned host copies, a stream and events
 * per device until the process ends; batched steps on one device take their
 * grouped part one at a time.
 * Errors: NQS_EINVAL (null context). */
int nqs_set_cg_grouping(nqs_ctx* ctx, int enable);

/* Name of kernel class k, or NULL. */
const char* nqs_profile_class_name(int k);

#ifdef __cplusplus
}
#endif

#endif /* NQS_H */
