// Host-side launchers of the libnqs kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace nqs {

// Derived per-parameter tables in the compute precision R (double for FP64,
// float otherwise):
//   Tt [N][Mw]  tanh(2 W_ji) at [i][j]  (site-major; sampler rows)
//   Tj [Mw][Nw] tanh(2 W_ji) at [j][i]  (hidden-major; local energies)
//   Ks [N][2]   site factor K_i(+1), K_i(-1) (FP64) or their logs (FP32)
//   Wa [Na][Mw] W~^T: W_ji at [i][j], b_j at [N][j] (theta contraction)
//   Whi, Wlo [Mw][Kb] BF16 two-term split of W~ (hidden-major; BF16 form only)
struct Tables {
    void* Tt;
    void* Tj;
    void* Ks;
    void* Wa;
    uint16_t* Whi;
    uint16_t* Wlo;
};

// Scalars and counters the CG kernels keep on the device (float64 slots).
struct CgScalars {
    double rr;        // r . r
    double rr0;       // f . f
    double pAp;       // p . A p
    double alpha;
    double beta;
    double tol2;      // tol^2 * f.f
    double wmean;     // mean of w in the current product
    double pad0;
    int32_t iters;    // iterations done
    int32_t done;     // converged or stopped
    int32_t maxiter;
    int32_t bad;      // non-finite scalar seen
    uint32_t counter[8];  // last-block counters
    // on-the-fly CG: set by the init kernel, so that the iteration kernels take
    // no per-iteration arguments (a batch of iterations can be replayed as is)
    double tol;       // relative residual tolerance
    double shift;     // diagonal shift
    double pp;        // p . p of the current direction
    double rr_prev;   // r . r of the previous iteration
    int32_t it;       // index of the next iteration (advanced by the update kernel)
    int32_t pad1;
};

// tables.hip
void launch_unpack(hipStream_t st, const Dims& d, const double* p, double* Pm, int P);
void launch_pack(hipStream_t st, const Dims& d, const double* Pm, double* p, int P);
void launch_mask(hipStream_t st, const Dims& d, double* V);
void launch_tables(hipStream_t st, const Dims& d, int prec, const double* Pm, const Tables& t);
void launch_init_chains(hipStream_t st, int N, int C, uint64_t seed, int sz0, int8_t* s);
void launch_zero(hipStream_t st, void* p, size_t bytes);

// theta.hip: t~ = tanh(S~ W~^T) for `rows` configurations (row stride N),
// written to dst1 (row stride Mw) and, if dst2 != null, to dst2 with row
// stride dst2_stride elements.
void launch_theta(hipStream_t st, const Dims& d, int prec, const Tables& t, const int8_t* s,
                  int rows, void* dst1, void* dst2, long dst2_stride);
// ln psi(s) (out: float64 for prec 0, float32 otherwise)
void launch_log_psi(hipStream_t st, const Dims& d, int prec, const double* Pm, const Tables& t,
                    const int8_t* s, long n, void* out);

// sampler.hip
struct SampleArgs {
    int C;                 // chains
    int K;                 // proposals in this launch
    int record;            // write the final configuration to rec (row stride rec_stride)
    uint64_t seed;
    uint64_t prop_base;    // global proposal index of the first proposal
    int8_t* s;             // [C][N] chain configurations (in/out)
    const void* tch;       // [C][Mw] tanh(theta) at the start of the launch
    int8_t* rec;           // recorded configuration destination
    long rec_stride;       // bytes between chains in rec
    uint8_t* acc_log;      // [C][log_stride] accept flags or null
    long log_stride;
    long log_offset;
    uint32_t* acc_count;   // [C] accepted counts (accumulated) or null
    int n_bonds;
    const int32_t* bonds;  // exchange rule
};
void launch_sample(hipStream_t st, const Dims& d, int prec, int rule, const Tables& t,
                   const SampleArgs& a);

// eloc.hip
struct HamDev {
    int kind;              // 0 TFIM, 1 Heisenberg
    int n_bonds;
    const int32_t* bonds;  // [n_bonds][2]
    const int8_t* sub;     // [N] or null
    double J, h;
};
void launch_eloc(hipStream_t st, const Dims& d, int prec, const Tables& t, const HamDev& H,
                 const int8_t* s, const void* tact, long n, double* out, size_t lds_limit);

// sr.hip
void launch_stats(hipStream_t st, const double* E, long n, double* out3);
void launch_center(hipStream_t st, const double* E, const double* stats, double scale, long n,
                   double* v);
int outer_chunk(const Dims& d, int prec, size_t lds_limit);
int outer_ksplit(long n, int chunk);
// part: [outer_ksplit(n, chunk)][Ma][Na]
void launch_outer(hipStream_t st, const Dims& d, int prec, const int8_t* s, const void* tact,
                  long n, const double* v, int v_mode, void* part, int chunk,
                  const CgScalars* sc);
void launch_reduce_outer(hipStream_t st, const Dims& d, int prec, const void* part, int ksplit,
                         const double* p, double shift, double* out, double* dpart,
                         CgScalars* sc, int mode);
void launch_cg_init(hipStream_t st, int total, const double* f, double* x, double* r, double* p,
                    double* dpart, CgScalars* sc, double tol, int maxiter, double shift);
// dense-form CG iteration after the product: dpart holds the product's npap
// partials of p.Ap, followed by room for the update's partials of r.r; with
// host_flag (pinned), the stop flag is also stored there
void launch_cg_update(hipStream_t st, int total, double* x, double* r, double* p,
                      const double* Ap, double* dpart, int npap, CgScalars* sc,
                      int32_t* host_flag = nullptr);
void launch_axpy_update(hipStream_t st, int total, double* x, const double* delta, double lr,
                        CgScalars* sc);

// qgt.hip: force and on-the-fly QGT products of one SR step, and CG
struct QgtBatch {
    void* Sp;        // augmented spins, sample-major: int8 [Nsp][Kq] (FP64) or FP4 [Nsp][Kq/2]
    int8_t* St;      // augmented spins, site-major: int8 [Kb][Nsp] (FP64) or FP4 [Kb][Nsp/2]
    void* Th;        // [Ma][Nsp] t~ hidden-major: double (FP64 path) or float
    float* Tf;       // BF16 forms: t~ in contraction-1 fragment order (Nsp * Ma floats)
    long Nsp;        // samples padded to a multiple of 512
    int kc;          // BF16 forms: samples per contraction-2 chunk (0 on the FP64 path)
    int ks;          // contraction-2 partial slots: chunks (BF16) or sample ranges (FP64)
    double* wpart;   // [qgt_nbw(n, prec)] block partials of sum w
};
long qgt_padded_samples(long n);
size_t qgt_th_bytes(const Dims& d, int prec, long Nsp);
int qgt_nbw(long n, int prec);
// activation rows to allocate for n samples (whole contraction-1 blocks)
long qgt_act_rows(long n);
int qgt_nbu(const Dims& d);
int qgt_nbr(const Dims& d);   // 64-entry blocks of a CG vector (the largest partial count)
int qgt_nbv(const Dims& d, int prec);  // CG update blocks = head partials per array
size_t qgt_spin_bytes(const Dims& d, int prec, long Nsp);  // bytes of Sp (and of St)
int qgt_ksplit(const QgtBatch& q);
// sets q.kc and q.ks for n samples (q.Nsp set) on a device with ncu CUs
void qgt_split(QgtBatch& q, const Dims& d, int prec, long n, int ncu);
int qgt_nbo(const Dims& d, const QgtBatch& q);  // p.G p partials (one per slot)
void launch_qgt_prepare(hipStream_t st, const Dims& d, int prec, const int8_t* s,
                        const void* tact, long n, const QgtBatch& q);
// bytes of a vector in the contraction-1 operand layout
size_t qgt_pop_bytes(const Dims& d, int prec);
// CG iteration, kernel 1: head (stop test, beta, p.p) + w = J r + beta w (in place)
void launch_qgt_w(hipStream_t st, const Dims& d, int prec, const QgtBatch& q, const void* tact,
                  long n, const void* Rop, double* w, const double* aux, CgScalars* sc);
// kernel 2 (and the force with v_mode 1): slot partials of J^T z
void launch_qgt_outer(hipStream_t st, const Dims& d, int prec, const QgtBatch& q, long n,
                      const double* v, int v_mode, void* part, double* papart,
                      const CgScalars* sc);
// force: sum of the slot partials
void launch_qgt_reduce(hipStream_t st, const Dims& d, int prec, const void* part, int ksplit,
                       const double* p, double shift, double* out, double* pap,
                       const CgScalars* sc, int cg);
// kernel 3: direction, product, x and r, head partials for the next iteration
void launch_qgt_update(hipStream_t st, const Dims& d, int prec, const QgtBatch& q,
                       const void* part, double* x, double* r, const double* p_old,
                       double* p_new, void* Rop, const double* papart, double* aux_next,
                       CgScalars* sc, int32_t* host_flag);
void launch_qgt_init(hipStream_t st, const Dims& d, int prec, const double* f, double* x,
                     double* r, double* p, double* p2, void* Rop, double* aux0, double* w, long n,
                     double tol, int maxiter, double shift, CgScalars* sc);

// Grouped on-the-fly CG iterations (BF16 forms): the three iteration kernels
// of up to CG_GROUP_MAX independent runs, one launch per kernel class (the
// head + contraction-1 blocks sized for the run with the most contraction
// waves; a smaller run's extra waves idle).  Each run keeps
// its own blocks and fixed-order sums, so its results are those of its own
// launches.  The table lives in device memory; cg_group_plan fills it.
constexpr int CG_GROUP_MAX = 32;
struct CgGroupRun {
    Dims d;
    long n, Nsp;
    const void* Sp;
    const void* St;
    const float* Tf;
    const void* Th;
    void* Rop;
    double* w;       // w = J v (and the contraction-2 source)
    double* wpart;   // contraction-1 block partials
    double* aux;     // head partials: two sets of 3 nbv, alternating with the iteration
    void* part;      // contraction-2 chunk partials
    double* papart;  // p . G p chunk partials
    double *x, *r, *p, *p2;  // p and p2 alternate as the old and new direction
    CgScalars* sc;
    int32_t* host_flag;  // pinned: the stop flag after the last iteration of a batch
    int nbv, nbw, ks;
    int nwc;  // contraction-1 waves of the run's own launch (set by cg_group_plan)
};
struct CgGroupTable {
    int nrun;
    // each run's first block in the launch of each class, ascending in table
    // order, INT_MAX past the last run (the contraction-1 launches, one per
    // block size, number their blocks on from one another)
    int first_w[CG_GROUP_MAX], first_o[CG_GROUP_MAX], first_u[CG_GROUP_MAX];
    CgGroupRun run[CG_GROUP_MAX];
};
// the launches of one grouped iteration
struct CgGroupPlan {
    int nw;  // contraction-1 launches (one): first block, blocks, block size
    int w_base[CG_GROUP_MAX], w_blocks[CG_GROUP_MAX], w_threads[CG_GROUP_MAX];
    int o_blocks, u_blocks;
    int u_sw;  // update: slot slabs per wave loaded up front (the largest the runs need)
};
// Fills in the block offsets (and each run's contraction-1 wave count) of the
// run entries of t (t.nrun of them, with their operands set).
void cg_group_plan(CgGroupTable& t, CgGroupPlan& plan);
// One grouped iteration; par = iteration & 1 (which direction buffer and head
// partial set is the old one); write_flag: the update stores each run's stop
// flag in its host_flag.
void launch_cg_group_iter(hipStream_t st, const CgGroupTable* t_dev, const CgGroupPlan& plan,
                          int par, int write_flag);

// dense.hip
void launch_jacobian_centred(hipStream_t st, const Dims& d, int prec, const int8_t* s,
                             const void* tact, long n, void* O, int P, long ld, double* cs,
                             double* scratch, size_t scratch_bytes, bool split);
void launch_jacobian(hipStream_t st, const Dims& d, int prec, const int8_t* s, const void* tact,
                     long n, void* O, int P, long ld);
// centre and scale the columns of O [n][ld] (first P); scratch (may be null)
// holds column-sum partials, up to 64 row slices of P doubles; split (FP32
// entries only): store each entry as the BF16 pair (hi << 16) | lo that the
// BF16 Gram reads
void launch_center_cols(hipStream_t st, int prec, void* O, long n, long ld, int P, double* cs,
                        double* scratch, size_t scratch_bytes, bool split);
int gram_tiles(int P);
void fill_gram_tiles(int P, int* host_tiles);
void launch_gram(hipStream_t st, int prec, const void* A, long n, long ld, int P, void* G,
                 const int* tiles, int ntiles);
// FP64 Gram over row slices (deterministic slice sum); slices from gram_slices,
// part: gram_part_bytes(ntiles, slices) of scratch (slices == 1: the plain kernel)
int gram_slices(int ntiles, long n);
size_t gram_part_bytes(int ntiles, int slices);
void launch_gram_sliced(hipStream_t st, const double* A, long n, long ld, int P, double* G,
                        const int* tiles, int ntiles, int slices, double* part);
int dense_matvec_blocks(int P);  // blocks (and p.Ap partials) of one dense product
// (G + shift I) v, the shift taken from sc
void launch_dense_matvec(hipStream_t st, int prec, const void* G, int P, long ld, const double* v,
                         double* out, double* dpart, CgScalars* sc);

// holo.hip: complex-parameter (holomorphic) RBM, complex FP64 (double2)
int h_max_hidden();
void launch_h_tables(hipStream_t st, int N, int M, const double2* p, double2* T, double2* K);
// tanh(theta) of `rows` configurations into t [rows][M] (and t2 with row stride t2_stride)
void launch_h_theta(hipStream_t st, int N, int M, const double2* p, const int8_t* s, long rows,
                    double2* t, double2* t2, long t2_stride);
void launch_h_log_psi(hipStream_t st, int N, int M, const double2* p, const int8_t* s, long n,
                      double2* out);
void launch_h_sample(hipStream_t st, int N, int M, const double2* T, const double2* K,
                     const SampleArgs& a, const double2* tch);
void launch_h_eloc(hipStream_t st, int N, int M, const double2* T, const double2* K,
                   const HamDev& H, const int8_t* s, const double2* tact, long n, double2* out);
void launch_h_stats(hipStream_t st, const double2* E, long n, double* out);
// scratch bytes the Jacobian embedding and the force need (slice partials)
size_t h_slice_bytes(int P);
void launch_h_jacobian(hipStream_t st, int N, int M, const int8_t* s, const double2* t, long n,
                       int P, double2* O);
// U [2 n8][ld] = [Re; Im] of (O - mean O) / sqrt(n), stacked, each half
// n8 = h_half_rows(n) rows (rows past n zero); mean: complex [P]
__host__ __device__ inline long h_half_rows(long n) { return (n + 7) / 8 * 8; }
void launch_h_jacobian_emb(hipStream_t st, int N, int M, const int8_t* s, const double2* t,
                           long n, int P, long ld, double* U, double2* mean, double* scratch);
// f [2P] = [Re | Im] of dJ^H (E - mean E) / sqrt(n), from U
void launch_h_force(hipStream_t st, const double* U, long n, long ld, int P, const double2* E,
                    const double* stats, double* f, double* scratch);
// A = Re G (G [P][ld]) and B = Im G (G + P ld) from U; tiles from fill_gram_tiles(P);
// part: h_gram_part_bytes(ntiles, slices) of scratch
int h_gram_slices(int ntiles, long n);
size_t h_gram_part_bytes(int ntiles, int slices);
void launch_h_gram(hipStream_t st, const double* U, long n, long ld, int P, const int* tiles,
                   int ntiles, int slices, double* part, double* G);
// (G + shift I) v for [[A, -B], [B, A]] (v, out: [re | im], 2P; shift from sc) and the block
// partials of v.(G + shift I) v (h_matvec_blocks(P) of them)
int h_matvec_blocks(int P);
void launch_h_matvec(hipStream_t st, const double* G, int P, long ld, const double* v,
                     double* out, double* dpart, CgScalars* sc);
// out = in + c x (+ c2 x2), x and x2 embedded [re | im], c complex
void launch_h_axpy(hipStream_t st, int P, const double2* in, double cr, double ci, const double* x,
                   double c2r, double c2i, const double* x2, double2* out);
void launch_h_split(hipStream_t st, int P, const double2* z, double* emb);
void launch_h_join(hipStream_t st, int P, const double* emb, double2* z);

// chol.hip: (A + shift I) x = f by an in-place blocked Cholesky of the FP64
// symmetric A [n][ld] (lower triangle read and overwritten by L), then the two
// triangular solves; bad (device int) set when a pivot is not positive; the CG
// scalars sc are set to those of a converged solve (no iterations) or bad
// (Yinv: chol_side_bytes(n) of scratch for the diagonal blocks' inverses)
size_t chol_side_bytes(int n);
// (y: n doubles of scratch; x must not alias f)
void launch_chol_solve(hipStream_t st, double* A, int n, long ld, double shift, const double* f,
                       double* x, int32_t* bad, double* Yinv, double* y, CgScalars* sc);
// holo.hip: the lower triangle of E = [[Re G, -Im G], [Im G, Re G]] ([2P][lde]) from
// Re G = G and Im G = G + P ld
void launch_h_embed(hipStream_t st, const double* G, int P, long ld, double* E, long lde);

// probe.hip: throughput probes (kind 0 FP32 FMA, 1 FP64 FMA, 2 FP32 exp, 3 FP64
// MFMA, 4 BF16 MFMA); launch_probe returns the work one launch does (flops, or
// exponentials for kind 2); sink: probe_sink_bytes() of device memory
size_t probe_sink_bytes();
double launch_probe(hipStream_t st, int kind, void* sink);

// symm.hip: symmetric RBM (alpha features over a site-permutation group G,
// expanded to the plain RBM with alpha |G| hidden units, hidden unit i |G| + g)
int symm_num_params(int N, int alpha, int vb, int hb);
// psym -> the plain RBM's packed parameters (out: N + M + M N doubles, biases as flagged)
void launch_symm_expand(hipStream_t st, int N, int G, int alpha, int vb, int hb,
                        const int32_t* perms, const double* psym, double* out);
// the plain force in the augmented [Ma][Na] layout -> the symmetric one (sums over G)
void launch_symm_tie(hipStream_t st, int N, int G, int alpha, int vb, int hb, int Na,
                     const int32_t* perms, const double* grad, double* out);
// O [n][ld] FP64 = d ln psi / d psym for n configurations s with activations t
// ([n][Mw], FP64 for prec 0, FP32 otherwise); columns past P_sym zero
void launch_symm_jacobian(hipStream_t st, int prec, int N, int G, int alpha, int vb, int hb,
                          int Mw, const int32_t* perms, const int8_t* s, const void* t, long n,
                          long ld, double* O);

}  // namespace nqs
