// C ABI of libnqs (declared in include/nqs.h): context state, workspace
// layout and the host-side orchestration of the kernels.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <set>
#include <vector>

#include "../../include/nqs.h"
#include "kernels.h"

using namespace nqs;

namespace {

constexpr size_t ALIGN = 256;

struct Buffers {
    double *Pm, *grad, *x, *r, *p, *p2, *Ap, *tmpv, *gacc;
    int32_t* bonds;
    int8_t* sub;
    Tables tab;
    int8_t* chains;
    void* tch;
    int8_t* samples;
    void* tsm;
    void* tx;
    double *eloc, *vvec, *wbuf, *stats, *dpart;
    QgtBatch q;
    double *rrp, *pap;
    void* Pop;
    uint32_t* acc_count;
    CgScalars* sc;
    void* part;
    // dense QGT
    void* O;
    void* G;
    double *colsum, *fp, *xp, *rp, *pp, *App;
    int* tiles;
    // complex (holomorphic) model: parameters (and a saved copy), tables,
    // activations of the chains, of the sample batch and of a local-energy
    // batch, local energies, Jacobian column means, the TDVP's first slope
    double2 *hp, *hp0, *hT, *hK, *htch, *htsm, *htx, *heloc, *hmean;
    double* hk1;
    double* psym;     // symmetric model: its parameters
    double* gpart;    // FP64 dense Gram: slice partials (when sliced)
    int32_t* cbad;    // Cholesky: pivot-not-positive flag
    double* cinv;     // Cholesky: inverses of the 32 x 32 diagonal blocks
    double* hE;       // complex + Cholesky: the real embedding of G
    int32_t* perms;   // symmetric model: the group, [G][N]
    double* hgp;  // complex: Gram slice partials
};

}  // namespace

struct CgRun;

struct nqs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // Hamiltonian
    int ham_kind = -1;
    int N = 0;
    std::vector<int32_t> bonds;
    std::vector<int8_t> sub;
    bool has_sub = false;
    double J = 0.0, h = 0.0;
    // model
    bool has_model = false;
    int M = 0, vb = 1, hb = 1, prec = 0;
    bool cplx = false;  // complex parameters (NQS_C128)
    long Plc = 0;       // complex: row stride of the stacked Jacobian U and of Re G, Im G
    int hS = 1;         // complex: row slices of the Gram
    int gS = 1;         // FP64 dense Gram (real, symmetric): row slices
    int dsolver = NQS_SOLVER_CG;  // how dense QGT systems are solved
    long Ple = 0;       // complex + Cholesky: row stride of the real embedding E
    int Pd = 0;         // size of the dense SR system: P, 2 P (real embedding) or P_sym
    // symmetric model (nqs_set_rbm_symm): M = alpha |G| hidden units of the plain
    // RBM it expands to; P stays that RBM's count, Psym the model's own
    bool symm = false;
    int alpha = 0, G = 0, Psym = 0;
    std::vector<int32_t> perms;
    Dims d{};
    size_t P = 0;
    // sampler
    bool has_sampler = false;
    int rule = 0, C = 0, S = 0, K = 0, sz0 = 0;
    uint64_t seed = 0;
    uint64_t prop = 0;
    int qgt = NQS_QGT_ONTHEFLY;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    Buffers b{};
    long Ns = 0, Bx = 0;
    int ksplit = 1, chunk = 256, ndpart = 1, Pld = 0, ntiles = 0;
    size_t lds_limit = 65536;
    int ncu = 256;  // compute units of the device
    long cg_iter = 0;
    double cg_tol = 1e-6;
    int cg_maxiter = 0;
    // state
    bool params_set = false, chains_dirty = true, have_samples = false, have_grad = false;
    double acceptance = 0.0;
    CgScalars* h_sc = nullptr;  // pinned
    int32_t* h_flag = nullptr;  // pinned [2]: CG stop flag after a batch of iterations
    hipEvent_t flag_ev[2] = {nullptr, nullptr};
    double* h_stats = nullptr;  // pinned [4]
    uint32_t* h_acc = nullptr;  // pinned [C]
    size_t h_acc_n = 0;
    // event profiler
    uint32_t prof_mask = 0;
    std::vector<hipEvent_t> ev;   // start/stop pairs
    std::vector<int> ev_class;
    size_t ev_used = 0;
    int64_t prof_count[NQS_PROF_CLASSES] = {};
    // a full batch of on-the-fly CG iterations captured as a HIP graph
    bool graphs = true;
    // the batched step may run this context's CG iterations in grouped launches
    bool grouping = true;
    hipGraphExec_t cg_graph = nullptr;
    hipGraphExec_t cg_graph_dense = nullptr;  // a batch of dense-form iterations
    hipStream_t cap_stream = nullptr;
    // a step issued by nqs_step_begin: 0 none, 1 in CG, 2 update issued, results
    // on their way to the host (step_ev marks their arrival)
    int step_phase = 0;
    nqs_step_cfg step_cfg{};
    CgRun* step_run = nullptr;
    hipEvent_t step_ev = nullptr;
    // device address of this GPU's static scratch (nqs_local_energy_noalloc)
    void* scratch_dev = nullptr;
};

namespace {

int fail(nqs_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

// Brackets the launches issued in its scope with a pair of HIP events when
// the kernel class is being profiled.
struct ProfScope {
    nqs_ctx* c;
    long slot = -1;
    ProfScope(nqs_ctx* ctx, int k) : c(ctx) {
        if (!((c->prof_mask >> k) & 1u)) return;
        if (c->ev_used + 2 > c->ev.size()) return;  // pool full: neither timed nor counted
        slot = (long)c->ev_used;
        c->ev_used += 2;
        c->ev_class[slot / 2] = k;
        c->prof_count[k] += 1;
        hipEventRecord(c->ev[slot], c->stream);
    }
    ~ProfScope() {
        if (slot >= 0) hipEventRecord(c->ev[slot + 1], c->stream);
    }
};
#define PROF(k) ProfScope prof_scope_(c, k)

#define HIPCHK(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ctx, NQS_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

int last_launch(nqs_ctx* c) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, NQS_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return NQS_OK;
}

size_t esize(int prec) { return prec == 0 ? 8 : 4; }

size_t layout_holo(nqs_ctx* c, char* base);

// Walk the workspace; with base == nullptr only the size is computed.
size_t layout(nqs_ctx* c, char* base) {
    if (c->cplx) return layout_holo(c, base);
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        off = (off + ALIGN - 1) / ALIGN * ALIGN;
        void* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const Dims& d = c->d;
    const size_t es = esize(c->prec);
    const size_t PV = (size_t)d.Ma * d.Na;
    const size_t PVX = PV > c->P ? PV : c->P;
    Buffers& b = c->b;
    b.Pm = (double*)take(8 * PV);
    b.grad = (double*)take(8 * PV);
    b.x = (double*)take(8 * PV);
    b.r = (double*)take(8 * PV);
    b.p = (double*)take(8 * PV);
    b.p2 = (double*)take(8 * PV);
    b.Ap = (double*)take(8 * PV);
    b.tmpv = (double*)take(8 * PVX);
    b.gacc = (double*)take(8 * PV);
    b.bonds = (int32_t*)take(8 * c->bonds.size() / 2 + 8);
    b.sub = (int8_t*)take((size_t)c->N + 16);
    b.tab.Tt = take(es * (size_t)d.N * d.Mw);
    b.tab.Tj = take(es * (size_t)d.Mw * d.Nw);
    b.tab.Ks = take(es * 2 * (size_t)d.N);
    b.tab.Wa = take(es * (size_t)d.Na * d.Mw);
    if (c->prec == 2) {
        b.tab.Whi = (uint16_t*)take(2 * (size_t)d.Kb * d.Mw);
        b.tab.Wlo = (uint16_t*)take(2 * (size_t)d.Kb * d.Mw);
    } else {
        b.tab.Whi = b.tab.Wlo = nullptr;
    }
    b.chains = (int8_t*)take((size_t)c->C * d.N);
    b.tch = take(es * (size_t)c->C * d.Mw);
    b.samples = (int8_t*)take((size_t)c->Ns * d.N);
    b.tsm = take(es * (size_t)qgt_act_rows(c->Ns) * d.Mw);
    b.tx = take(es * (size_t)c->Bx * d.Mw);
    b.eloc = (double*)take(8 * (size_t)c->Bx);
    // per-sample vectors the contractions read in whole 512-sample chunks
    const long Nvec = c->Bx > qgt_padded_samples(c->Ns) ? c->Bx : qgt_padded_samples(c->Ns);
    b.vvec = (double*)take(8 * (size_t)Nvec);
    b.wbuf = (double*)take(8 * (size_t)Nvec);
    b.stats = (double*)take(8 * 8);
    b.dpart = (double*)take(8 * (size_t)c->ndpart);
    b.acc_count = (uint32_t*)take(4 * (size_t)c->C);
    b.sc = (CgScalars*)take(sizeof(CgScalars));
    b.cbad = (int32_t*)take(16);
    b.hE = nullptr;
    b.cinv = c->dsolver == NQS_SOLVER_CHOLESKY ? (double*)take(chol_side_bytes(c->Pd)) : nullptr;
    {
        const long Nsp = qgt_padded_samples(c->Ns);
        b.q.Nsp = Nsp;
        qgt_split(b.q, d, c->prec, c->Ns, c->ncu);
        // FP64: int8 spins; BF16 forms: one FP4 code per spin
        b.q.Sp = take(qgt_spin_bytes(d, c->prec, Nsp));
        b.q.St = (int8_t*)take(qgt_spin_bytes(d, c->prec, Nsp));
        b.q.Th = take(qgt_th_bytes(d, c->prec, Nsp));
        b.q.Tf = c->prec == 0 ? nullptr : (float*)take(4 * (size_t)Nsp * d.Ma);
        b.q.wpart = (double*)take(8 * (size_t)qgt_nbw(Nsp, c->prec));
        // CG head partials (r.r, r.p, p.p), one set per iteration parity
        b.rrp = (double*)take(8 * 2 * 3 * (size_t)qgt_nbr(d));
        b.pap = (double*)take(8 * (size_t)qgt_nbo(d, b.q));   // p.G p partials
        b.Pop = take(qgt_pop_bytes(d, c->prec));               // r, contraction-1 layout
        const size_t ks = (size_t)(c->ksplit > b.q.ks ? c->ksplit : b.q.ks);
        b.part = take(es * ks * PV);
    }
    if (c->symm) {
        b.psym = (double*)take(8 * (size_t)c->Psym);
        b.perms = (int32_t*)take(4 * c->perms.size());
    } else {
        b.psym = nullptr;
        b.perms = nullptr;
    }
    if (c->qgt == NQS_QGT_JACOBIAN_DENSE) {
        // (a symmetric model's Jacobian and Gram are FP64, P_sym columns)
        const size_t des = c->symm ? 8 : es;
        b.O = take(des * (size_t)c->Ns * c->Pld);
        b.G = take(des * (size_t)c->Pd * c->Pld);
        b.colsum = (double*)take(8 * (size_t)c->Pld);
        b.gpart = c->gS > 1 ? (double*)take(gram_part_bytes(c->ntiles, c->gS)) : nullptr;
        b.fp = (double*)take(8 * (size_t)c->Pld);
        b.xp = (double*)take(8 * (size_t)c->Pld);
        b.rp = (double*)take(8 * (size_t)c->Pld);
        b.pp = (double*)take(8 * (size_t)c->Pld);
        b.App = (double*)take(8 * (size_t)c->Pld);
        b.tiles = (int*)take(8 * (size_t)c->ntiles);
    } else {
        b.O = b.G = nullptr;
        b.colsum = b.fp = b.xp = b.rp = b.pp = b.App = nullptr;
        b.tiles = nullptr;
    }
    return (off + ALIGN - 1) / ALIGN * ALIGN;
}

// The complex model's workspace: its own parameter, table and activation
// buffers; chains, samples, scalars and the dense-QGT buffers as in the real
// layout, with the embedded Jacobian Y [2 Ns][Pld] in O and the Gram matrix
// of the 2 P-dimensional embedded system in G (whose buffer first holds the
// slice partials of the column sums and of the force).
size_t layout_holo(nqs_ctx* c, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        off = (off + ALIGN - 1) / ALIGN * ALIGN;
        void* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const size_t P = c->P, N = (size_t)c->N, M = (size_t)c->M, C = (size_t)c->C;
    const size_t Ns = (size_t)c->Ns, Bx = (size_t)c->Bx, Pld = (size_t)c->Pld;
    Buffers& b = c->b;
    b = Buffers{};
    b.hp = (double2*)take(16 * P);
    b.hp0 = (double2*)take(16 * P);
    b.hT = (double2*)take(16 * N * M);
    b.hK = (double2*)take(16 * 2 * N);
    b.bonds = (int32_t*)take(8 * c->bonds.size() / 2 + 8);
    b.sub = (int8_t*)take(N + 16);
    b.chains = (int8_t*)take(C * N);
    b.htch = (double2*)take(16 * C * M);
    b.samples = (int8_t*)take(Ns * N);
    b.htsm = (double2*)take(16 * Ns * M);
    b.htx = (double2*)take(16 * Bx * M);
    b.heloc = (double2*)take(16 * (Ns > Bx ? Ns : Bx));
    b.stats = (double*)take(8 * 8);
    b.dpart = (double*)take(8 * (size_t)c->ndpart);
    b.acc_count = (uint32_t*)take(4 * C);
    b.sc = (CgScalars*)take(sizeof(CgScalars));
    const size_t Plc = (size_t)c->Plc;
    b.O = take(8 * 2 * (size_t)h_half_rows((long)Ns) * Plc);  // U: two halves
    const size_t gb = 8 * 2 * P * Plc, sb = h_slice_bytes((int)P);
    b.G = take(gb > sb ? gb : sb);
    b.hgp = (double*)take(h_gram_part_bytes(c->ntiles, c->hS));
    b.hmean = (double2*)take(16 * P);
    b.fp = (double*)take(8 * Pld);
    b.xp = (double*)take(8 * Pld);
    b.rp = (double*)take(8 * Pld);
    b.pp = (double*)take(8 * Pld);
    b.App = (double*)take(8 * Pld);
    b.hk1 = (double*)take(8 * Pld);
    b.cbad = (int32_t*)take(16);
    b.hE = c->dsolver == NQS_SOLVER_CHOLESKY ? (double*)take(8 * 2 * P * (size_t)c->Ple) : nullptr;
    b.cinv = c->dsolver == NQS_SOLVER_CHOLESKY ? (double*)take(chol_side_bytes(c->Pd)) : nullptr;
    b.tiles = (int*)take(8 * (size_t)c->ntiles);
    return (off + ALIGN - 1) / ALIGN * ALIGN;
}

bool configured(const nqs_ctx* c) { return c->ham_kind >= 0 && c->has_model && c->has_sampler; }

void derive(nqs_ctx* c) {
    Dims& d = c->d;
    d.N = c->N;
    d.M = c->M;
    d.Na = round_up(c->N + 1, 16);
    d.Ma = round_up(c->M + 1, 16);
    // the sampler keeps 64 * QMAX activations per chain (QMAX = QM rounded up
    // to a power of two); rows are padded that far with zero table entries
    int qmax = 1;
    while (qmax < (c->M + 63) / 64) qmax *= 2;
    d.Mw = d.Ma > 64 * qmax ? d.Ma : 64 * qmax;
    d.Nw = round_up(c->N, 64);
    d.Kb = round_up(d.Na, 32);
    d.Kq = round_up(d.Na, 128);
    d.QM = (c->M + 63) / 64;
    d.vb = c->vb;
    d.hb = c->hb;
    c->P = (size_t)(c->vb ? c->N : 0) + (c->hb ? c->M : 0) + (size_t)c->M * c->N;
    c->cplx = c->prec == NQS_C128;
    if (c->symm) c->Psym = symm_num_params(c->N, c->alpha, c->vb, c->hb);
    c->Pd = (int)(c->cplx ? 2 * c->P : c->symm ? (size_t)c->Psym : c->P);
    if (c->has_sampler) {
        c->Ns = (long)c->C * c->S;
        c->Bx = c->Ns > 1024 ? c->Ns : 1024;
        c->chunk = outer_chunk(d, c->prec, c->lds_limit);
        c->ksplit = outer_ksplit(c->Bx, c->chunk);
        c->Pld = round_up(c->Pd, 128);
        c->ntiles = gram_tiles(c->Pd);
        if (c->cplx) {  // Re G and Im G are P x P
            c->Plc = round_up((long)c->P, 128);
            c->ntiles = gram_tiles((int)c->P);
            c->hS = h_gram_slices(c->ntiles, c->Ns);
        }
        c->gS = (!c->cplx && (c->symm || c->prec == 0)) ? gram_slices(c->ntiles, c->Ns) : 1;
        c->Ple = round_up(2 * (long)c->P, 128);
        long nd = (long)d.Ma * d.Na / 256 + 2;
        const long nd2 = c->Bx / 64 + 2, nd3 = (long)c->Pd / 4 + 2;
        if (nd2 > nd) nd = nd2;
        if (nd3 > nd) nd = nd3;
        c->ndpart = (int)nd;
    }
}

void invalidate_binding(nqs_ctx* c) {
    c->bound = false;
    c->ws = nullptr;
    c->ws_bytes = 0;
    c->have_samples = c->have_grad = false;
}

HamDev ham_dev(const nqs_ctx* c) {
    HamDev H;
    H.kind = c->ham_kind;
    H.n_bonds = (int)(c->bonds.size() / 2);
    H.bonds = c->b.bonds;
    H.sub = c->has_sub ? c->b.sub : nullptr;
    H.J = c->J;
    H.h = c->h;
    return H;
}

int need_bound(nqs_ctx* c) {
    if (!c) return NQS_EINVAL;
    if (!c->bound) return fail(c, NQS_ESTATE, "no workspace bound");
    if (!c->params_set) return fail(c, NQS_ESTATE, "parameters not set");
    return NQS_OK;
}

int set_device(nqs_ctx* c) {
    HIPCHK(c, hipSetDevice(c->device));
    return NQS_OK;
}

// tanh(theta) of the chains' current configurations
void refresh_chains(nqs_ctx* c) {
    if (!c->chains_dirty) return;
    {
        PROF(NQS_PROF_THETA);
        launch_theta(c->stream, c->d, c->prec, c->b.tab, c->b.chains, c->C, c->b.tch, nullptr, 0);
    }
    c->chains_dirty = false;
}

int check_bonds(nqs_ctx* c, int n_sites, int n_bonds, const int32_t* bonds) {
    if (n_sites < 2 || n_bonds < 1 || !bonds) return fail(c, NQS_EINVAL, "bad lattice size");
    for (int k = 0; k < n_bonds; ++k) {
        const int a = bonds[2 * k], b2 = bonds[2 * k + 1];
        if (a < 0 || a >= n_sites || b2 < 0 || b2 >= n_sites || a == b2)
            return fail(c, NQS_EINVAL, "bond " + std::to_string(k) + " has a bad site index");
    }
    return NQS_OK;
}

int set_ham(nqs_ctx* c, int kind, int n_sites, int n_bonds, const int32_t* bonds, double J,
            double h, const int8_t* sub) {
    int st = check_bonds(c, n_sites, n_bonds, bonds);
    if (st) return st;
    if (!std::isfinite(J) || !std::isfinite(h)) return fail(c, NQS_EINVAL, "non-finite coupling");
    if (c->has_model && n_sites != c->N) {
        c->has_model = false;
        c->has_sampler = false;
        c->params_set = false;
    }
    c->ham_kind = kind;
    c->N = n_sites;
    c->bonds.assign(bonds, bonds + 2 * (size_t)n_bonds);
    c->J = J;
    c->h = h;
    c->has_sub = sub != nullptr;
    c->sub.assign((size_t)n_sites, 0);
    if (sub)
        for (int i = 0; i < n_sites; ++i) c->sub[i] = sub[i] ? 1 : 0;
    if (c->bound) {
        // same sizes: refresh the device copy in place
        if (c->has_model && layout(c, nullptr) <= c->ws_bytes) {
            layout(c, c->ws);
            HIPCHK(c, hipMemcpyAsync(c->b.bonds, c->bonds.data(), 4 * c->bonds.size(),
                                     hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->b.sub, c->sub.data(), c->sub.size(), hipMemcpyHostToDevice,
                                     c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        } else {
            invalidate_binding(c);
        }
    }
    return NQS_OK;
}

int enqueue_scalars(nqs_ctx* c) {
    HIPCHK(c, hipMemcpyAsync(c->h_sc, c->b.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, c->stream));
    return NQS_OK;
}
int sync_scalars(nqs_ctx* c) {
    int st = enqueue_scalars(c);
    if (st) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NQS_OK;
}

int cg_check_interval() {
    static int v = [] {
        const char* e = std::getenv("NQS_CG_CHECK");
        int x = e ? std::atoi(e) : 0;
        return x > 0 ? x : 10;
    }();
    return v;
}

// ---- staged pieces of the hot path (asynchronous unless noted) -------------

void issue_sample(nqs_ctx* c, int n_discard, uint8_t* accept_log) {
    refresh_chains(c);
    SampleArgs a{};
    a.C = c->C;
    a.K = c->K;
    a.seed = c->seed;
    a.s = c->b.chains;
    a.tch = c->b.tch;
    a.n_bonds = (int)(c->bonds.size() / 2);
    a.bonds = c->b.bonds;
    for (int q = 0; q < n_discard; ++q) {
        a.prop_base = c->prop;
        a.record = 0;
        launch_sample(c->stream, c->d, c->prec, c->rule, c->b.tab, a);
        c->prop += (uint64_t)c->K;
        {
        PROF(NQS_PROF_THETA);
        launch_theta(c->stream, c->d, c->prec, c->b.tab, c->b.chains, c->C, c->b.tch, nullptr, 0);
    }
    }
    launch_zero(c->stream, c->b.acc_count, 4 * (size_t)c->C);
    a.acc_count = c->b.acc_count;
    a.acc_log = accept_log;
    a.log_stride = (long)c->S * c->K;
    const size_t es = esize(c->prec);
    for (int q = 0; q < c->S; ++q) {
        a.prop_base = c->prop;
        a.record = 1;
        a.rec = c->b.samples + (size_t)q * c->d.N;
        a.rec_stride = (long)c->S * c->d.N;
        a.log_offset = (long)q * c->K;
        {
            PROF(NQS_PROF_SAMPLE);
            launch_sample(c->stream, c->d, c->prec, c->rule, c->b.tab, a);
        }
        c->prop += (uint64_t)c->K;
        {
            PROF(NQS_PROF_THETA);
            launch_theta(c->stream, c->d, c->prec, c->b.tab, c->b.chains, c->C, c->b.tch,
                         (char*)c->b.tsm + es * (size_t)q * c->d.Mw, (long)c->S * c->d.Mw);
        }
    }
    c->have_samples = true;
    c->have_grad = false;
}

void issue_energy_grad(nqs_ctx* c) {
    const long n = c->Ns;
    {
        PROF(NQS_PROF_ELOC);
        launch_eloc(c->stream, c->d, c->prec, c->b.tab, ham_dev(c), c->b.samples, c->b.tsm, n,
                    c->b.eloc, c->lds_limit);
    }
    {
        PROF(NQS_PROF_STATS);
        launch_stats(c->stream, c->b.eloc, n, c->b.stats);
        launch_center(c->stream, c->b.eloc, c->b.stats, 2.0 / (double)n, n, c->b.vvec);
    }
    {
        PROF(NQS_PROF_PREPARE);
        launch_qgt_prepare(c->stream, c->d, c->prec, c->b.samples, c->b.tsm, n, c->b.q);
    }
    {
        PROF(NQS_PROF_OUTER);
        launch_qgt_outer(c->stream, c->d, c->prec, c->b.q, n, c->b.vvec, 1, c->b.part, c->b.pap,
                         c->b.sc);
    }
    {
        PROF(NQS_PROF_REDUCE);
        launch_qgt_reduce(c->stream, c->d, c->prec, c->b.part, qgt_ksplit(c->b.q), nullptr, 0.0,
                          c->b.grad, nullptr, c->b.sc, 0);
    }
    c->have_grad = true;
}

// Host copies of the energy statistics, the accept counters and the CG scalars are
// enqueued with enqueue_* and used by take_* after the stream has been synchronised,
// so that a caller that needs several of them waits for the device once.
int enqueue_stats(nqs_ctx* c) {
    HIPCHK(c, hipMemcpyAsync(c->h_stats, c->b.stats, 4 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    return NQS_OK;
}
int take_stats(nqs_ctx* c, nqs_stats* E) {
    if (E) {
        E->mean = c->h_stats[0];
        E->variance = c->h_stats[1];
        E->error = c->h_stats[2];
        E->acceptance = c->acceptance;
    }
    if (!std::isfinite(c->h_stats[0])) return fail(c, NQS_ENUMERIC, "non-finite energy");
    return NQS_OK;
}
int read_stats(nqs_ctx* c, nqs_stats* E) {
    int st = enqueue_stats(c);
    if (st) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return take_stats(c, E);
}

int enqueue_acceptance(nqs_ctx* c) {
    HIPCHK(c, hipMemcpyAsync(c->h_acc, c->b.acc_count, 4 * (size_t)c->C, hipMemcpyDeviceToHost,
                             c->stream));
    return NQS_OK;
}
int take_acceptance(nqs_ctx* c) {
    double acc = 0.0;
    for (int k = 0; k < c->C; ++k) acc += c->h_acc[k];
    c->acceptance = acc / ((double)c->C * c->S * c->K);
    return NQS_OK;
}
int read_acceptance(nqs_ctx* c) {
    int st = enqueue_acceptance(c);
    if (st) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return take_acceptance(c);
}

// dense Jacobian form: build G once for this batch and set up CG in packed space
void issue_dense_setup(nqs_ctx* c, double tol, int maxiter, double shift) {
    const int P = (int)c->P;
    {
        PROF(NQS_PROF_JACOBIAN);
        // (the Gram matrix's buffer is free until the Gram is formed: column-sum partials)
        launch_jacobian_centred(c->stream, c->d, c->prec, c->b.samples, c->b.tsm, c->Ns, c->b.O,
                                P, c->Pld, c->b.colsum, (double*)c->b.G,
                                esize(c->prec) * (size_t)c->P * c->Pld, c->prec == 2);
    }
    {
        PROF(NQS_PROF_GRAM);
        if (c->prec == 0)
            launch_gram_sliced(c->stream, (const double*)c->b.O, c->Ns, c->Pld, P,
                               (double*)c->b.G, c->b.tiles, c->ntiles, c->gS, c->b.gpart);
        else
            launch_gram(c->stream, c->prec, c->b.O, c->Ns, c->Pld, P, c->b.G, c->b.tiles,
                        c->ntiles);
    }
    launch_pack(c->stream, c->d, c->b.grad, c->b.fp, P);
    launch_cg_init(c->stream, P, c->b.fp, c->b.xp, c->b.rp, c->b.pp, c->b.dpart, c->b.sc, tol,
                   maxiter, shift);
}

void issue_cg_init(nqs_ctx* c, double tol, int maxiter, double shift) {
    c->cg_iter = 0;
    c->cg_tol = tol;
    c->cg_maxiter = maxiter;
    launch_qgt_init(c->stream, c->d, c->prec, c->b.grad, c->b.x, c->b.r, c->b.p, c->b.p2,
                    c->b.Pop, c->b.rrp, c->b.wbuf, c->Ns, tol, maxiter, shift, c->b.sc);
}

// CG iterations.  On-the-fly form, three kernels per iteration: the head
// (convergence test on the residual left by iteration it - 1, beta) with
// w = J r + beta w; the chunk partials of J^T z; the update, which forms
// p_new = r + beta p_old (the direction alternates between two buffers, the
// head partials too) and updates x and r.
// Dense form: product, update, direction (the shift is in the scalars).
// With host_flag, the last iteration stores the stop flag there.
void issue_cg_iters(nqs_ctx* c, int kind, double shift, int iters, int32_t* host_flag = nullptr) {
    const Dims& d = c->d;
    const int nbv = qgt_nbv(d, c->prec);
    for (int it = 0; it < iters; ++it) {
        if (kind == NQS_QGT_ONTHEFLY) {
            const long k = c->cg_iter;
            double* p_old = (k & 1) ? c->b.p2 : c->b.p;
            double* p_new = (k & 1) ? c->b.p : c->b.p2;
            double* aux_cur = c->b.rrp + (k & 1) * 3 * nbv;
            double* aux_next = c->b.rrp + ((k + 1) & 1) * 3 * nbv;
            c->cg_iter += 1;
            {
                PROF(NQS_PROF_QGT_W);
                launch_qgt_w(c->stream, d, c->prec, c->b.q, c->b.tsm, c->Ns, c->b.Pop, c->b.wbuf,
                             aux_cur, c->b.sc);
            }
            {
                PROF(NQS_PROF_OUTER);
                launch_qgt_outer(c->stream, d, c->prec, c->b.q, c->Ns, c->b.wbuf, 0, c->b.part,
                                 c->b.pap, c->b.sc);
            }
            {
                PROF(NQS_PROF_REDUCE);
                launch_qgt_update(c->stream, d, c->prec, c->b.q, c->b.part, c->b.x, c->b.r, p_old,
                                  p_new, c->b.Pop, c->b.pap, aux_next, c->b.sc,
                                  it + 1 == iters ? host_flag : nullptr);
            }
        } else {
            {
                PROF(NQS_PROF_DENSE_MV);
                if (c->cplx)
                    launch_h_matvec(c->stream, (const double*)c->b.G, (int)c->P, c->Plc, c->b.pp,
                                    c->b.App, c->b.dpart, c->b.sc);
                else
                    launch_dense_matvec(c->stream, c->symm ? 0 : c->prec, c->b.G, c->Pd, c->Pld,
                                        c->b.pp, c->b.App, c->b.dpart, c->b.sc);
            }
            {
                PROF(NQS_PROF_CGVEC);
                launch_cg_update(c->stream, c->Pd, c->b.xp, c->b.rp, c->b.pp, c->b.App, c->b.dpart,
                                 c->cplx ? h_matvec_blocks((int)c->P) : dense_matvec_blocks(c->Pd),
                                 c->b.sc, it + 1 == iters ? host_flag : nullptr);
            }
        }
    }
}

// delta (internal layout) is in b.x after this
void issue_finish_solve(nqs_ctx* c, int kind) {
    if (kind == NQS_QGT_JACOBIAN_DENSE) launch_unpack(c->stream, c->d, c->b.xp, c->b.x, (int)c->P);
}

void issue_update(nqs_ctx* c, double lr) {
    {
        PROF(NQS_PROF_UPDATE);
        launch_axpy_update(c->stream, c->d.Ma * c->d.Na, c->b.Pm, c->b.x, lr, c->b.sc);
        launch_tables(c->stream, c->d, c->prec, c->b.Pm, c->b.tab);
    }
    c->chains_dirty = true;
    c->have_grad = false;
    c->have_samples = false;  // the held batch's activations belong to the old parameters
}

int sr_status(nqs_ctx* c, nqs_sr_info* info) {
    const CgScalars& s = *c->h_sc;
    if (info) {
        info->iterations = s.iters;
        info->converged = (s.rr <= s.tol2) ? 1 : 0;
        info->rel_residual = s.rr0 > 0 ? std::sqrt(s.rr / s.rr0) : 0.0;
    }
    if (s.bad) return fail(c, NQS_ENUMERIC, "non-finite value in the SR solve or update");
    if (!(s.rr <= s.tol2)) return fail(c, NQS_ENOTCONV, "CG reached maxiter before tolerance");
    return NQS_OK;
}

void drop_graphs(nqs_ctx* c) {
    if (c->cg_graph) hipGraphExecDestroy(c->cg_graph);
    c->cg_graph = nullptr;
    if (c->cg_graph_dense) hipGraphExecDestroy(c->cg_graph_dense);
    c->cg_graph_dense = nullptr;
}

// Records one batch of `every` on-the-fly iterations (starting at an even
// iteration, so the alternating buffers line up) as a graph.
int capture_batch(nqs_ctx* c, int kind, double shift, int every) {
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t run = c->stream;
    const long it0 = c->cg_iter;
    c->stream = c->cap_stream;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        issue_cg_iters(c, kind, shift, every, &c->h_flag[0]);
        e = hipStreamEndCapture(c->cap_stream, &graph);
    }
    c->stream = run;
    c->cg_iter = it0;
    hipGraphExec_t& g = kind == NQS_QGT_ONTHEFLY ? c->cg_graph : c->cg_graph_dense;
    if (e == hipSuccess) e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    if (e != hipSuccess) {
        g = nullptr;
        return fail(c, NQS_EDEVICE, std::string("CG graph capture: ") + hipGetErrorString(e));
    }
    return NQS_OK;
}

// kernel classes of the on-the-fly CG iterations
constexpr uint32_t CG_CLASSES = (1u << NQS_PROF_QGT_W) | (1u << NQS_PROF_OUTER) |
                                (1u << NQS_PROF_REDUCE) | (1u << NQS_PROF_CGVEC) |
                                (1u << NQS_PROF_DENSE_MV);

// Issues CG iterations in batches and reads the stop flag of each batch while
// the next batch is already queued, so the device never waits for the host.
// Iterations issued after the stop return at once (every CG kernel tests the
// flag first).  Full batches are replayed from one captured graph per form
// (the iteration kernels take their scalars from the device; the last one of
// a batch stores the stop flag in pinned host memory) unless CG kernel
// classes are being timed, which needs one event pair per launch and batches
// of one iteration.  One CgRun drives one context; the batched step drives
// several side by side.
}  // namespace

struct CgRun {
    nqs_ctx* c = nullptr;
    int kind = 0, every = 1, limit = 0;
    double shift = 0.0;
    bool use_graphs = false, stop = false;
    int launched = 0, issued = 0, checked = 0;

    void init(nqs_ctx* ctx, int k, double sh, int maxiter) {
        c = ctx;
        kind = k;
        shift = sh;
        // while CG kernels are timed, the stop flag is read after every iteration
        // so that almost no launch after the stop is timed
        every = (c->prof_mask & CG_CLASSES) ? 1 : cg_check_interval();
        // the on-the-fly form tests convergence at the start of an iteration
        limit = kind == NQS_QGT_ONTHEFLY ? maxiter + 1 : maxiter;
        use_graphs = c->graphs && every % 2 == 0 && !(c->prof_mask & CG_CLASSES);
    }
    bool finished() const { return stop || (checked >= issued && launched >= limit); }
    int issue_batch() {
        const int k = (limit - launched) < every ? (limit - launched) : every;
        const int slot = issued & 1;
        // (the on-the-fly form alternates buffers: its graph starts on an even iteration)
        if (use_graphs && k == every && (kind != NQS_QGT_ONTHEFLY || c->cg_iter % 2 == 0)) {
            hipGraphExec_t& g = kind == NQS_QGT_ONTHEFLY ? c->cg_graph : c->cg_graph_dense;
            if (!g) {
                const int st = capture_batch(c, kind, shift, every);
                if (st) return st;
            }
            HIPCHK(c, hipGraphLaunch(g, c->stream));
            c->cg_iter += every;
        } else {
            issue_cg_iters(c, kind, shift, k, &c->h_flag[0]);
        }
        launched += k;
        HIPCHK(c, hipEventRecord(c->flag_ev[slot], c->stream));
        ++issued;
        return NQS_OK;
    }
    // keep up to `depth` batches queued (a lone context: two, so the device never
    // waits for the host; contexts run side by side: one each, the others' work
    // fills the device and fewer iterations are queued past a context's stop)
    int top_up(int depth = 2) {
        while (!stop && launched < limit && issued - checked < depth) {
            const int st = issue_batch();
            if (st) return st;
        }
        return NQS_OK;
    }
    // read the stop flag of the oldest unchecked batch; without `block`, only
    // if that batch has finished (progress tells whether it was read)
    int poll(bool block, bool& progress) {
        progress = false;
        if (checked >= issued) return NQS_OK;
        const int slot = checked & 1;
        if (block) {
            HIPCHK(c, hipEventSynchronize(c->flag_ev[slot]));
        } else {
            const hipError_t e = hipEventQuery(c->flag_ev[slot]);
            if (e == hipErrorNotReady) return NQS_OK;
            HIPCHK(c, e);
        }
        // the batch's last iteration stored the flag in word 0 (a later batch may
        // already have overwritten it with a value just as valid: the flag only
        // goes from 0 to 1 within a solve)
        stop = c->h_flag[0] != 0;
        ++checked;
        progress = true;
        return NQS_OK;
    }
};

// ---- grouped CG iterations of the batched step -----------------------------
// The on-the-fly CG of several small BF16-form contexts on one device, one
// launch per kernel class per iteration for all of them (cg_group_plan), on a
// stream of the library's own.  Per device the library keeps up to
// CG_GROUP_SLOTS slots (two descriptor tables, their pinned host copies, a
// stream, events) until the process ends; one batched step at a time uses a
// device's slots.  The tables sit in a static device array (no device
// allocation): every GPU holds its own copy, and host code uses the address
// hipGetSymbolAddress returns on that device, never the array's name.
constexpr int CG_GROUP_SLOTS = 8;
static __device__ __align__(256) CgGroupTable group_tables[2 * CG_GROUP_SLOTS];

namespace {

// Contexts join a group when one CG iteration's contractions are small enough
// for launch overhead to dominate their own launches: samples x augmented
// hidden rows x site extent at most this (2^28, a few microseconds of work).
constexpr double CG_GROUP_WORK = 268435456.0;
bool group_small(const nqs_ctx* c) {
    return (double)c->Ns * c->d.Ma * c->d.Kq <= CG_GROUP_WORK;
}

struct GroupSlot {
    CgGroupTable* dev[2] = {nullptr, nullptr};
    CgGroupTable* host[2] = {nullptr, nullptr};  // pinned
    hipEvent_t copy_ev[2] = {nullptr, nullptr};  // after each table's upload
    hipStream_t stream = nullptr;
    hipEvent_t flag_ev[2] = {nullptr, nullptr};
    hipEvent_t done_ev = nullptr;
};
struct GroupPool {
    std::mutex m;
    CgGroupTable* tables = nullptr;  // device address of group_tables on this device
    std::vector<std::unique_ptr<GroupSlot>> slots;
};

GroupPool& group_pool(int device) {
    static std::mutex gm;
    static std::map<int, std::unique_ptr<GroupPool>> pools;
    std::lock_guard<std::mutex> l(gm);
    std::unique_ptr<GroupPool>& p = pools[device];
    if (!p) p.reset(new GroupPool);
    return *p;
}

// slot k of the pool (created on first use, the device current); null on
// failure or past CG_GROUP_SLOTS
GroupSlot* group_slot(GroupPool& pool, size_t k, std::string& err) {
    if (k >= (size_t)CG_GROUP_SLOTS) {
        err = "grouped CG: no free group slot";
        return nullptr;
    }
    if (!pool.tables) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(group_tables)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            err = "grouped CG set-up: no address for the group tables";
            return nullptr;
        }
        pool.tables = (CgGroupTable*)ptr;
    }
    while (pool.slots.size() <= k) {
        std::unique_ptr<GroupSlot> s(new GroupSlot);
        hipError_t e = hipSuccess;
        const size_t slot = pool.slots.size();
        for (int i = 0; i < 2 && e == hipSuccess; ++i) {
            s->dev[i] = pool.tables + 2 * slot + i;
            e = hipHostMalloc((void**)&s->host[i], sizeof(CgGroupTable), hipHostMallocDefault);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&s->copy_ev[i], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        for (int i = 0; i < 2 && e == hipSuccess; ++i)
            e = hipEventCreateWithFlags(&s->flag_ev[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->done_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            err = std::string("grouped CG set-up: ") + hipGetErrorString(e);
            return nullptr;  // (what was created stays with the process)
        }
        pool.slots.push_back(std::move(s));
    }
    return pool.slots[k].get();
}

}  // namespace

// Drives the CG iterations of its members in lock-step: batches of `every`
// grouped iterations, the members' stop flags read as batches finish (up to
// two batches queued).  A member whose flag says it has stopped leaves the
// table from the next batch issued on (the table is rebuilt in the slot's
// other buffer; batches already queued still read the old one, and their
// launches return at once for that member).
struct CgGroup {
    GroupSlot* s = nullptr;
    std::vector<nqs_ctx*> all;      // every member (the streams to release)
    std::vector<nqs_ctx*> members;  // those still iterating
    CgGroupPlan plan{};
    int cur = 0;  // table buffer the next batch reads
    int every = 1, limit = 0;
    bool stop = false;
    int launched = 0, issued = 0, checked = 0;
    std::string err;

    bool ok(hipError_t e, const char* what) {
        if (e == hipSuccess) return true;
        err = std::string(what) + ": " + hipGetErrorString(e);
        return false;
    }
    // fills table buffer cur from members and queues its upload
    bool upload() {
        hipError_t e = hipEventSynchronize(s->copy_ev[cur]);  // (its previous upload is done)
        if (!ok(e, "grouped CG table")) return false;
        CgGroupTable& t = *s->host[cur];
        t.nrun = (int)members.size();
        for (int r = 0; r < t.nrun; ++r) {
            const nqs_ctx* c = members[r];
            const Buffers& b = c->b;
            CgGroupRun& R = t.run[r];
            std::memset(&R, 0, sizeof(R));
            R.d = c->d;
            R.n = c->Ns;
            R.Nsp = b.q.Nsp;
            R.Sp = b.q.Sp;
            R.St = b.q.St;
            R.Tf = b.q.Tf;
            R.Th = b.q.Th;
            R.Rop = b.Pop;
            R.w = b.wbuf;
            R.wpart = b.q.wpart;
            R.aux = b.rrp;
            R.part = b.part;
            R.papart = b.pap;
            R.x = b.x;
            R.r = b.r;
            R.p = b.p;
            R.p2 = b.p2;
            R.sc = b.sc;
            R.host_flag = &c->h_flag[0];
            R.nbv = qgt_nbv(c->d, c->prec);
            R.nbw = qgt_nbw(c->Ns, c->prec);
            R.ks = qgt_ksplit(b.q);
        }
        cg_group_plan(t, plan);
        e = hipMemcpyAsync(s->dev[cur], s->host[cur], sizeof(CgGroupTable),
                           hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipEventRecord(s->copy_ev[cur], s->stream);
        return ok(e, "grouped CG table");
    }
    // cfg_limit: the largest number of iterations any member may launch
    bool start(int cfg_limit) {
        all = members;
        every = cg_check_interval();
        limit = cfg_limit;
        // the group's stream waits for each member's CG set-up (its flag_ev[0],
        // recorded after the set-up was issued)
        hipError_t e = hipStreamSynchronize(s->stream);  // (the slot's last use is over)
        for (nqs_ctx* c : members)
            if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, c->flag_ev[0], 0);
        return ok(e, "grouped CG start") && upload();
    }
    bool finished() const { return stop || (checked >= issued && launched >= limit); }
    bool issue_batch() {
        const int k = (limit - launched) < every ? (limit - launched) : every;
        for (int i = 0; i < k; ++i)
            launch_cg_group_iter(s->stream, s->dev[cur], plan, (launched + i) & 1, i + 1 == k);
        launched += k;
        if (!ok(hipGetLastError(), "grouped CG launch")) return false;
        if (!ok(hipEventRecord(s->flag_ev[issued & 1], s->stream), "grouped CG event"))
            return false;
        ++issued;
        return true;
    }
    bool top_up(int depth) {
        while (!stop && launched < limit && issued - checked < depth)
            if (!issue_batch()) return false;
        return true;
    }
    // as CgRun::poll; CG has stopped when every member's flag says so
    bool poll(bool block, bool& progress) {
        progress = false;
        if (checked >= issued) return true;
        hipEvent_t ev = s->flag_ev[checked & 1];
        if (block) {
            if (!ok(hipEventSynchronize(ev), "grouped CG wait")) return false;
        } else {
            const hipError_t e = hipEventQuery(ev);
            if (e == hipErrorNotReady) return true;
            if (!ok(e, "grouped CG query")) return false;
        }
        ++checked;
        progress = true;
        std::vector<nqs_ctx*> left;
        for (nqs_ctx* c : members)
            if (c->h_flag[0] == 0) left.push_back(c);
        stop = left.empty();
        if (stop || left.size() == members.size()) return true;
        members.swap(left);
        cur ^= 1;
        return upload();
    }
    // every member's stream waits for the group's work
    bool finish() {
        hipError_t e = hipEventRecord(s->done_ev, s->stream);
        for (nqs_ctx* c : all)
            if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, s->done_ev, 0);
        return ok(e, "grouped CG finish");
    }
};

namespace {

int run_cg(nqs_ctx* c, int kind, double shift, int maxiter) {
    CgRun r;
    r.init(c, kind, shift, maxiter);
    if (r.limit <= 0) return NQS_OK;
    int st = r.issue_batch();
    if (st) return st;
    while (!r.finished()) {
        st = r.top_up();
        if (st) return st;
        bool progress;
        st = r.poll(true, progress);
        if (st) return st;
    }
    return NQS_OK;
}

int default_maxiter(const nqs_ctx* c, int maxiter) {
    if (maxiter > 0) return maxiter;
    return c->Pd < 10000 ? c->Pd : 10000;
}

// ---- the complex (holomorphic) model ----------------------------------------
size_t param_doubles(const nqs_ctx* c) {
    return c->cplx ? 2 * c->P : c->symm ? (size_t)c->Psym : c->P;
}

int h_check(nqs_ctx* c) {
    if (c->ham_kind != 0) return fail(c, NQS_EINVAL, "complex models take the TFIM");
    if (c->has_sampler && c->rule != NQS_RULE_LOCAL)
        return fail(c, NQS_EINVAL, "complex models take the local rule");
    return NQS_OK;
}

void h_tables(nqs_ctx* c) { launch_h_tables(c->stream, c->N, c->M, c->b.hp, c->b.hT, c->b.hK); }

void h_refresh_chains(nqs_ctx* c) {
    if (!c->chains_dirty) return;
    {
        PROF(NQS_PROF_THETA);
        launch_h_theta(c->stream, c->N, c->M, c->b.hp, c->b.chains, c->C, c->b.htch, nullptr, 0);
    }
    c->chains_dirty = false;
}

// n_discard unrecorded segments, then S recorded ones (as issue_sample); the
// activations are recomputed from the configurations after every segment
void h_issue_sample(nqs_ctx* c, int n_discard, int n_record, uint8_t* accept_log) {
    h_refresh_chains(c);
    SampleArgs a{};
    a.C = c->C;
    a.K = c->K;
    a.seed = c->seed;
    a.s = c->b.chains;
    for (int q = 0; q < n_discard; ++q) {
        a.prop_base = c->prop;
        a.record = 0;
        {
            PROF(NQS_PROF_SAMPLE);
            launch_h_sample(c->stream, c->N, c->M, c->b.hT, c->b.hK, a, c->b.htch);
        }
        c->prop += (uint64_t)c->K;
        {
            PROF(NQS_PROF_THETA);
            launch_h_theta(c->stream, c->N, c->M, c->b.hp, c->b.chains, c->C, c->b.htch, nullptr, 0);
        }
    }
    if (!n_record) return;
    launch_zero(c->stream, c->b.acc_count, 4 * (size_t)c->C);
    a.acc_count = c->b.acc_count;
    a.acc_log = accept_log;
    a.log_stride = (long)c->S * c->K;
    for (int q = 0; q < c->S; ++q) {
        a.prop_base = c->prop;
        a.record = 1;
        a.rec = c->b.samples + (size_t)q * c->N;
        a.rec_stride = (long)c->S * c->N;
        a.log_offset = (long)q * c->K;
        {
            PROF(NQS_PROF_SAMPLE);
            launch_h_sample(c->stream, c->N, c->M, c->b.hT, c->b.hK, a, c->b.htch);
        }
        c->prop += (uint64_t)c->K;
        {
            PROF(NQS_PROF_THETA);
            launch_h_theta(c->stream, c->N, c->M, c->b.hp, c->b.chains, c->C, c->b.htch,
                           c->b.htsm + (size_t)q * c->M, (long)c->S * c->M);
        }
    }
    c->have_samples = true;
    c->have_grad = false;
}

// local energies, statistics, the embedded Jacobian and the embedded force
void h_issue_energy_grad(nqs_ctx* c) {
    const long n = c->Ns;
    {
        PROF(NQS_PROF_ELOC);
        launch_h_eloc(c->stream, c->N, c->M, c->b.hT, c->b.hK, ham_dev(c), c->b.samples, c->b.htsm,
                      n, c->b.heloc);
    }
    {
        PROF(NQS_PROF_STATS);
        launch_h_stats(c->stream, c->b.heloc, n, c->b.stats);
    }
    {
        PROF(NQS_PROF_JACOBIAN);
        launch_h_jacobian_emb(c->stream, c->N, c->M, c->b.samples, c->b.htsm, n, (int)c->P, c->Plc,
                              (double*)c->b.O, c->b.hmean, (double*)c->b.G);
        launch_h_force(c->stream, (const double*)c->b.O, n, c->Plc, (int)c->P, c->b.heloc,
                       c->b.stats, c->b.fp, (double*)c->b.G);
    }
    c->have_grad = true;
}

// the Gram matrix of the embedded system and its CG solve (x in xp)
int h_issue_solve(nqs_ctx* c, double diag_shift, double tol, int maxiter) {
    const int mi = default_maxiter(c, maxiter);
    {
        PROF(NQS_PROF_GRAM);
        launch_h_gram(c->stream, (const double*)c->b.O, c->Ns, c->Plc, (int)c->P, c->b.tiles,
                      c->ntiles, c->hS, c->b.hgp, (double*)c->b.G);
    }
    if (c->dsolver == NQS_SOLVER_CHOLESKY) {  // on the real embedding, size 2P
        PROF(NQS_PROF_CGVEC);
        launch_h_embed(c->stream, (const double*)c->b.G, (int)c->P, c->Plc, c->b.hE, c->Ple);
        launch_chol_solve(c->stream, c->b.hE, c->Pd, c->Ple, diag_shift, c->b.fp, c->b.xp,
                          c->b.cbad, c->b.cinv, c->b.rp, c->b.sc);
        return NQS_OK;
    }
    launch_cg_init(c->stream, c->Pd, c->b.fp, c->b.xp, c->b.rp, c->b.pp, c->b.dpart, c->b.sc, tol,
                   mi, diag_shift);
    return run_cg(c, NQS_QGT_JACOBIAN_DENSE, diag_shift, mi);
}

// new parameters: the tables follow; the chains' activations and the held batch
// belong to the old ones
void h_params_changed(nqs_ctx* c) {
    h_tables(c);
    c->chains_dirty = true;
    c->have_grad = false;
    c->have_samples = false;
}

// ---- the symmetric model ------------------------------------------------------
// new symmetric parameters: the plain RBM they expand to, its tables; chain
// activations and the held batch belong to the old ones
void s_params_changed(nqs_ctx* c) {
    launch_symm_expand(c->stream, c->N, c->G, c->alpha, c->vb, c->hb, c->b.perms, c->b.psym,
                       c->b.tmpv);
    launch_unpack(c->stream, c->d, c->b.tmpv, c->b.Pm, (int)c->P);
    launch_tables(c->stream, c->d, c->prec, c->b.Pm, c->b.tab);
    c->chains_dirty = true;
    c->have_grad = false;
    c->have_samples = false;
}

// the tied Jacobian of the held batch (centred, scaled), its Gram matrix and the
// CG solve of (S + eps I) x = f (x in xp; f in fp from the tied force)
int s_issue_solve(nqs_ctx* c, double diag_shift, double tol, int maxiter) {
    if (c->Ns > 65535)
        return fail(c, NQS_EINVAL, "the symmetric model's dense QGT takes at most 65535 samples");
    const int mi = default_maxiter(c, maxiter);
    {
        PROF(NQS_PROF_JACOBIAN);
        launch_symm_jacobian(c->stream, c->prec, c->N, c->G, c->alpha, c->vb, c->hb, c->d.Mw,
                             c->b.perms, c->b.samples, c->b.tsm, c->Ns, c->Pld, (double*)c->b.O);
        launch_center_cols(c->stream, 0, c->b.O, c->Ns, c->Pld, c->Psym, c->b.colsum,
                           (double*)c->b.G, 8 * (size_t)c->Pd * c->Pld, false);
    }
    {
        PROF(NQS_PROF_GRAM);
        launch_gram_sliced(c->stream, (const double*)c->b.O, c->Ns, c->Pld, c->Psym,
                           (double*)c->b.G, c->b.tiles, c->ntiles, c->gS, c->b.gpart);
    }
    if (c->dsolver == NQS_SOLVER_CHOLESKY) {
        PROF(NQS_PROF_CGVEC);
        launch_chol_solve(c->stream, (double*)c->b.G, c->Psym, c->Pld, diag_shift, c->b.fp, c->b.xp,
                          c->b.cbad, c->b.cinv, c->b.rp, c->b.sc);
        return NQS_OK;
    }
    launch_cg_init(c->stream, c->Psym, c->b.fp, c->b.xp, c->b.rp, c->b.pp, c->b.dpart, c->b.sc, tol,
                   mi, diag_shift);
    return run_cg(c, NQS_QGT_JACOBIAN_DENSE, diag_shift, mi);
}

__global__ void k_f32_to_f64(const float* a, double* b, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) b[e] = (double)a[e];
}
__global__ void k_f64_to_f32(const double* a, float* b, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) b[e] = (float)a[e];
}
__global__ void k_check_finite(const double* a, long n, int* flag) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n && !isfinite(a[e])) *flag = 1;
}

}  // namespace

// Static scratch of nqs_local_energy_noalloc, for callers that cannot
// allocate device memory: the hidden activations tanh(theta) of the batch.
// Every GPU the library runs on holds its own copy from module load until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol): kernels get the device address
// that hipGetSymbolAddress returns for the current device, looked up once per
// device when a context is created there.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the static scratch on `device`, which must be current.
void* scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_dev[device] = ptr;
    }
    return g_scratch_dev[device];
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int nqs_create(nqs_ctx** out, int device, void* hip_stream) {
    if (!out) return NQS_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return NQS_EINVAL;
    nqs_ctx* c = new nqs_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
        lds > 0)
        c->lds_limit = (size_t)lds;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        ncu > 0)
        c->ncu = ncu;
    if (hipSetDevice(device) != hipSuccess ||
        hipHostMalloc((void**)&c->h_sc, sizeof(CgScalars), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_stats, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_flag, 2 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->flag_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->flag_ev[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->step_ev, hipEventDisableTiming) != hipSuccess ||
        !(c->scratch_dev = scratch_address(device))) {
        nqs_destroy(c);
        return NQS_EDEVICE;
    }
    *out = c;
    return NQS_OK;
}

void nqs_destroy(nqs_ctx* c) {
    if (!c) return;
    if (c->stream) hipStreamSynchronize(c->stream);
    if (c->h_sc) hipHostFree(c->h_sc);
    if (c->h_stats) hipHostFree(c->h_stats);
    if (c->h_flag) hipHostFree(c->h_flag);
    for (auto& e : c->flag_ev)
        if (e) hipEventDestroy(e);
    if (c->step_ev) hipEventDestroy(c->step_ev);
    delete c->step_run;
    if (c->h_acc) hipHostFree(c->h_acc);
    for (auto& e : c->ev) hipEventDestroy(e);
    drop_graphs(c);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    delete c;
}

const char* nqs_last_error(const nqs_ctx* c) { return c ? c->err.c_str() : "null context"; }

int nqs_set_stream(nqs_ctx* c, void* hip_stream) {
    if (!c) return NQS_EINVAL;
    if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream));
    c->stream = (hipStream_t)hip_stream;
    return NQS_OK;
}

int nqs_set_tfim(nqs_ctx* c, int n_sites, int n_bonds, const int32_t* bonds, double J, double h) {
    if (!c) return NQS_EINVAL;
    return set_ham(c, 0, n_sites, n_bonds, bonds, J, h, nullptr);
}

int nqs_set_heisenberg(nqs_ctx* c, int n_sites, int n_bonds, const int32_t* bonds, double J,
                       const int8_t* sublattice) {
    if (!c) return NQS_EINVAL;
    return set_ham(c, 1, n_sites, n_bonds, bonds, J, 0.0, sublattice);
}

int nqs_set_rbm(nqs_ctx* c, int n_hidden, int visible_bias, int hidden_bias, nqs_precision prec) {
    if (!c) return NQS_EINVAL;
    if (c->ham_kind < 0) return fail(c, NQS_ESTATE, "set a Hamiltonian first");
    if (n_hidden < 1 || n_hidden > 2048) return fail(c, NQS_EINVAL, "n_hidden must be in [1, 2048]");
    if (prec < NQS_FP64 || prec > NQS_C128) return fail(c, NQS_EINVAL, "bad precision");
    if (c->N > 4096) return fail(c, NQS_EINVAL, "at most 4096 sites");
    if (prec == NQS_C128) {
        if (!visible_bias || !hidden_bias)
            return fail(c, NQS_EINVAL, "complex models keep both biases");
        if (n_hidden > h_max_hidden())
            return fail(c, NQS_EINVAL, "complex models take at most " +
                                           std::to_string(h_max_hidden()) + " hidden units");
        if (c->ham_kind != 0) return fail(c, NQS_EINVAL, "complex models take the TFIM");
        c->qgt = NQS_QGT_JACOBIAN_DENSE;
    }
    c->M = n_hidden;
    c->vb = visible_bias ? 1 : 0;
    c->hb = hidden_bias ? 1 : 0;
    c->prec = (int)prec;
    c->symm = false;
    c->perms.clear();
    c->has_model = true;
    c->params_set = false;
    derive(c);
    invalidate_binding(c);
    return NQS_OK;
}

int nqs_set_rbm_symm(nqs_ctx* c, int n_perms, const int32_t* perms, int alpha, int visible_bias,
                     int hidden_bias, nqs_precision prec) {
    if (!c) return NQS_EINVAL;
    if (c->ham_kind < 0) return fail(c, NQS_ESTATE, "set a Hamiltonian first");
    if (prec < NQS_FP64 || prec > NQS_BF16)
        return fail(c, NQS_EINVAL, "symmetric models take FP64, FP32 or BF16");
    if (n_perms < 1 || !perms || alpha < 1) return fail(c, NQS_EINVAL, "bad group or alpha");
    if ((long)alpha * n_perms > 2048)
        return fail(c, NQS_EINVAL, "alpha |G| (the hidden units) must be at most 2048");
    if (c->N > 4096) return fail(c, NQS_EINVAL, "at most 4096 sites");
    const int N = c->N;
    std::vector<int32_t> P(perms, perms + (size_t)n_perms * N);
    std::set<std::vector<int32_t>> rows;
    for (int g = 0; g < n_perms; ++g) {
        std::vector<int32_t> r(P.begin() + (size_t)g * N, P.begin() + (size_t)(g + 1) * N);
        std::vector<char> seen(N, 0);
        for (int k = 0; k < N; ++k) {
            if (r[k] < 0 || r[k] >= N || seen[r[k]])
                return fail(c, NQS_EINVAL, "row " + std::to_string(g) + " is not a permutation");
            seen[r[k]] = 1;
            if (g == 0 && r[k] != k) return fail(c, NQS_EINVAL, "row 0 must be the identity");
        }
        if (!rows.insert(r).second) return fail(c, NQS_EINVAL, "repeated permutation");
    }
    std::vector<int32_t> comp(N);
    for (int g = 0; g < n_perms; ++g)
        for (int h = 0; h < n_perms; ++h) {
            for (int k = 0; k < N; ++k) comp[k] = P[(size_t)g * N + P[(size_t)h * N + k]];
            if (!rows.count(comp)) return fail(c, NQS_EINVAL, "the permutations do not form a group");
        }
    c->perms.swap(P);
    c->G = n_perms;
    c->alpha = alpha;
    c->symm = true;
    c->M = alpha * n_perms;
    c->vb = visible_bias ? 1 : 0;
    c->hb = hidden_bias ? 1 : 0;
    c->prec = (int)prec;
    c->qgt = NQS_QGT_JACOBIAN_DENSE;
    c->has_model = true;
    c->params_set = false;
    derive(c);
    invalidate_binding(c);
    return NQS_OK;
}

size_t nqs_num_params(const nqs_ctx* c) {
    return (c && c->has_model) ? (c->symm ? (size_t)c->Psym : c->P) : 0;
}

int nqs_set_sampler(nqs_ctx* c, nqs_rule rule, int n_chains, int samples_per_chain,
                    int sweep_size, uint64_t seed, int total_sz_zero) {
    if (!c) return NQS_EINVAL;
    if (!c->has_model) return fail(c, NQS_ESTATE, "set the RBM first");
    if (rule != NQS_RULE_LOCAL && rule != NQS_RULE_EXCHANGE) return fail(c, NQS_EINVAL, "bad rule");
    if (n_chains < 1 || samples_per_chain < 1 || sweep_size < 1)
        return fail(c, NQS_EINVAL, "chains, samples and sweep size must be positive");
    if ((long)n_chains * samples_per_chain > (1L << 26)) return fail(c, NQS_EINVAL, "too many samples");
    if (total_sz_zero && (c->N % 2)) return fail(c, NQS_EINVAL, "total_sz_zero needs even n_sites");
    if (c->cplx && rule != NQS_RULE_LOCAL)
        return fail(c, NQS_EINVAL, "complex models take the local rule");
    c->rule = (int)rule;
    c->C = n_chains;
    c->S = samples_per_chain;
    c->K = sweep_size;
    c->seed = seed;
    c->sz0 = total_sz_zero ? 1 : 0;
    c->has_sampler = true;
    derive(c);
    invalidate_binding(c);
    if (c->h_acc) hipHostFree(c->h_acc);
    c->h_acc = nullptr;
    if (hipHostMalloc((void**)&c->h_acc, 4 * (size_t)n_chains, hipHostMallocDefault) != hipSuccess)
        return fail(c, NQS_EDEVICE, "pinned host buffer");
    return NQS_OK;
}

int nqs_set_qgt(nqs_ctx* c, nqs_qgt kind) {
    if (!c) return NQS_EINVAL;
    if (kind != NQS_QGT_ONTHEFLY && kind != NQS_QGT_JACOBIAN_DENSE)
        return fail(c, NQS_EINVAL, "bad QGT kind");
    if (c->cplx && kind != NQS_QGT_JACOBIAN_DENSE)
        return fail(c, NQS_EINVAL, "complex models use the dense holomorphic QGT");
    if (c->symm && kind != NQS_QGT_JACOBIAN_DENSE)
        return fail(c, NQS_EINVAL, "symmetric models use the dense QGT");
    if (c->qgt != (int)kind) {
        c->qgt = (int)kind;
        invalidate_binding(c);
    }
    return NQS_OK;
}

int nqs_set_dense_solver(nqs_ctx* c, nqs_dense_solver solver) {
    if (!c) return NQS_EINVAL;
    if (solver != NQS_SOLVER_CG && solver != NQS_SOLVER_CHOLESKY)
        return fail(c, NQS_EINVAL, "bad solver");
    if (solver == NQS_SOLVER_CHOLESKY && c->has_model) {
        if (!c->cplx && !c->symm && c->prec != 0)
            return fail(c, NQS_EINVAL, "the Cholesky solve takes the FP64 dense QGT");
        if (c->cplx && 2 * c->P > 32768)
            return fail(c, NQS_EINVAL, "the Cholesky solve of a complex model takes P <= 16384");
    }
    if (c->dsolver != (int)solver) {
        c->dsolver = (int)solver;
        invalidate_binding(c);  // the solver's buffers (and a complex model's embedding)
    }
    return NQS_OK;
}

size_t nqs_workspace_bytes(const nqs_ctx* c) {
    if (!c || !configured(c)) return 0;
    nqs_ctx tmp = *c;
    tmp.h_sc = nullptr;
    tmp.h_stats = nullptr;
    tmp.h_acc = nullptr;
    const size_t n = layout(&tmp, nullptr);
    return n;
}

int nqs_bind_workspace(nqs_ctx* c, void* dev_ptr, size_t bytes) {
    if (!c) return NQS_EINVAL;
    if (!configured(c)) return fail(c, NQS_ESTATE, "Hamiltonian, RBM and sampler must be set");
    if (c->cplx) {
        const int st = h_check(c);
        if (st) return st;
    }
    const size_t need = layout(c, nullptr);
    if (!dev_ptr || bytes < need)
        return fail(c, NQS_ENOMEM, "workspace needs " + std::to_string(need) + " bytes");
    if ((uintptr_t)dev_ptr % ALIGN) return fail(c, NQS_EINVAL, "workspace must be 256-byte aligned");
    int st = set_device(c);
    if (st) return st;
    drop_graphs(c);  // captured against the previous buffers
    c->ws = (char*)dev_ptr;
    c->ws_bytes = bytes;
    layout(c, c->ws);
    launch_zero(c->stream, c->ws, need);
    HIPCHK(c, hipMemcpyAsync(c->b.bonds, c->bonds.data(), 4 * c->bonds.size(), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->b.sub, c->sub.data(), c->sub.size(), hipMemcpyHostToDevice,
                             c->stream));
    if (c->symm)
        HIPCHK(c, hipMemcpyAsync(c->b.perms, c->perms.data(), 4 * c->perms.size(),
                                 hipMemcpyHostToDevice, c->stream));
    if (c->qgt == NQS_QGT_JACOBIAN_DENSE) {
        std::vector<int> t(2 * (size_t)c->ntiles);
        fill_gram_tiles(c->cplx ? (int)c->P : c->Pd, t.data());
        HIPCHK(c, hipMemcpyAsync(c->b.tiles, t.data(), 4 * t.size(), hipMemcpyHostToDevice,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    launch_init_chains(c->stream, c->N, c->C, c->seed, c->sz0, c->b.chains);
    c->prop = 0;
    c->bound = true;
    c->params_set = false;
    c->chains_dirty = true;
    c->have_samples = c->have_grad = false;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return last_launch(c);
}

int nqs_set_params(nqs_ctx* c, const double* p, int on_device) {
    if (!c) return NQS_EINVAL;
    if (!c->bound) return fail(c, NQS_ESTATE, "no workspace bound");
    if (!p) return fail(c, NQS_EINVAL, "null parameters");
    int st = set_device(c);
    if (st) return st;
    const size_t np = param_doubles(c);
    std::vector<double> h(np);
    if (on_device) {
        HIPCHK(c, hipMemcpyAsync(h.data(), p, 8 * np, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        std::memcpy(h.data(), p, 8 * np);
    }
    for (size_t k = 0; k < np; ++k)
        if (!std::isfinite(h[k])) return fail(c, NQS_ENUMERIC, "non-finite parameter");
    if (c->cplx) {
        HIPCHK(c, hipMemcpyAsync(c->b.hp, h.data(), 8 * np, hipMemcpyHostToDevice, c->stream));
        const bool held = c->have_samples;
        h_params_changed(c);
        if (held) {  // activations of the held batch follow the new parameters
            launch_h_theta(c->stream, c->N, c->M, c->b.hp, c->b.samples, c->Ns, c->b.htsm,
                           nullptr, 0);
            c->have_samples = true;
        }
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->params_set = true;
        return last_launch(c);
    }
    if (c->symm) {  // the symmetric parameters, expanded to the plain RBM's
        HIPCHK(c, hipMemcpyAsync(c->b.psym, h.data(), 8 * np, hipMemcpyHostToDevice, c->stream));
        launch_symm_expand(c->stream, c->N, c->G, c->alpha, c->vb, c->hb, c->b.perms, c->b.psym,
                           c->b.tmpv);
    } else {
        HIPCHK(c, hipMemcpyAsync(c->b.tmpv, h.data(), 8 * c->P, hipMemcpyHostToDevice, c->stream));
    }
    launch_unpack(c->stream, c->d, c->b.tmpv, c->b.Pm, (int)c->P);
    launch_tables(c->stream, c->d, c->prec, c->b.Pm, c->b.tab);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->params_set = true;
    c->chains_dirty = true;
    c->have_grad = false;
    if (c->have_samples)  // activations of the held batch follow the new parameters
        launch_theta(c->stream, c->d, c->prec, c->b.tab, c->b.samples, (int)c->Ns, c->b.tsm,
                     nullptr, 0);
    return last_launch(c);
}

int nqs_get_params(nqs_ctx* c, double* p, int on_device) {
    int st = need_bound(c);
    if (st) return st;
    if (!p) return fail(c, NQS_EINVAL, "null output");
    if (c->cplx) {
        HIPCHK(c, hipMemcpyAsync(p, c->b.hp, 16 * c->P,
                                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return last_launch(c);
    }
    if (c->symm) {
        HIPCHK(c, hipMemcpyAsync(p, c->b.psym, 8 * (size_t)c->Psym,
                                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return last_launch(c);
    }
    launch_pack(c->stream, c->d, c->b.Pm, c->b.tmpv, (int)c->P);
    HIPCHK(c, hipMemcpyAsync(p, c->b.tmpv, 8 * c->P,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return last_launch(c);
}

int nqs_reset_chains(nqs_ctx* c) {
    if (!c) return NQS_EINVAL;
    if (!c->bound) return fail(c, NQS_ESTATE, "no workspace bound");
    launch_init_chains(c->stream, c->N, c->C, c->seed, c->sz0, c->b.chains);
    c->prop = 0;
    c->chains_dirty = true;
    return last_launch(c);
}

int nqs_get_chains(nqs_ctx* c, int8_t* out, int on_device) {
    if (!c) return NQS_EINVAL;
    if (!c->bound || !out) return fail(c, NQS_ESTATE, "no workspace bound or null output");
    HIPCHK(c, hipMemcpyAsync(out, c->b.chains, (size_t)c->C * c->N,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NQS_OK;
}

int nqs_set_chains(nqs_ctx* c, const int8_t* in, int on_device) {
    if (!c) return NQS_EINVAL;
    if (!c->bound || !in) return fail(c, NQS_ESTATE, "no workspace bound or null input");
    HIPCHK(c, hipMemcpyAsync(c->b.chains, in, (size_t)c->C * c->N,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->chains_dirty = true;
    return NQS_OK;
}

uint64_t nqs_proposal_count(const nqs_ctx* c) { return c ? c->prop : 0; }

int nqs_get_state(nqs_ctx* c, void* blob, size_t* bytes) {
    int st = need_bound(c);
    if (st) return st;
    if (!bytes) return fail(c, NQS_EINVAL, "null size");
    const size_t need = 32 + 8 * param_doubles(c) + (size_t)c->C * c->N;
    if (!blob) {
        *bytes = need;
        return NQS_OK;
    }
    if (*bytes < need) return fail(c, NQS_EINVAL, "blob too small");
    char* o = (char*)blob;
    const uint64_t hdr[4] = {0x4E51535354415445ull, (uint64_t)c->P,
                             ((uint64_t)c->C << 32) | (uint32_t)c->N, c->prop};
    std::memcpy(o, hdr, 32);
    st = nqs_get_params(c, (double*)(o + 32), 0);
    if (st) return st;
    st = nqs_get_chains(c, (int8_t*)(o + 32 + 8 * param_doubles(c)), 0);
    if (st) return st;
    *bytes = need;
    return NQS_OK;
}

int nqs_set_state(nqs_ctx* c, const void* blob, size_t bytes) {
    if (!c) return NQS_EINVAL;
    if (!c->bound) return fail(c, NQS_ESTATE, "no workspace bound");
    const size_t need = 32 + 8 * param_doubles(c) + (size_t)c->C * c->N;
    if (!blob || bytes < need) return fail(c, NQS_EINVAL, "blob too small");
    uint64_t hdr[4];
    std::memcpy(hdr, blob, 32);
    if (hdr[0] != 0x4E51535354415445ull || hdr[1] != c->P ||
        hdr[2] != (((uint64_t)c->C << 32) | (uint32_t)c->N))
        return fail(c, NQS_EINVAL, "blob does not match this configuration");
    const char* in = (const char*)blob;
    int st = nqs_set_params(c, (const double*)(in + 32), 0);
    if (st) return st;
    st = nqs_set_chains(c, (const int8_t*)(in + 32 + 8 * param_doubles(c)), 0);
    if (st) return st;
    c->prop = hdr[3];
    c->have_samples = c->have_grad = false;
    return NQS_OK;
}

int nqs_sample(nqs_ctx* c, int n_discard_segments, int8_t* samples_out, uint8_t* accept_log,
               double* acceptance) {
    int st = need_bound(c);
    if (st) return st;
    if (n_discard_segments < 0) return fail(c, NQS_EINVAL, "negative discard count");
    st = set_device(c);
    if (st) return st;
    if (c->cplx) h_issue_sample(c, n_discard_segments, 1, accept_log);
    else issue_sample(c, n_discard_segments, accept_log);
    if (samples_out)
        HIPCHK(c, hipMemcpyAsync(samples_out, c->b.samples, (size_t)c->Ns * c->N,
                                 hipMemcpyDeviceToDevice, c->stream));
    st = last_launch(c);
    if (st) return st;
    if (acceptance) {
        st = read_acceptance(c);
        if (st) return st;
        *acceptance = c->acceptance;
    }
    return NQS_OK;
}

int nqs_thermalize(nqs_ctx* c, int n_segments) {
    int st = need_bound(c);
    if (st) return st;
    if (n_segments < 0) return fail(c, NQS_EINVAL, "negative segment count");
    st = set_device(c);
    if (st) return st;
    if (c->cplx) {
        h_issue_sample(c, n_segments, 0, nullptr);
        return last_launch(c);
    }
    refresh_chains(c);
    SampleArgs a{};
    a.C = c->C;
    a.K = c->K;
    a.seed = c->seed;
    a.s = c->b.chains;
    a.tch = c->b.tch;
    a.n_bonds = (int)(c->bonds.size() / 2);
    a.bonds = c->b.bonds;
    for (int q = 0; q < n_segments; ++q) {
        a.prop_base = c->prop;
        {
            PROF(NQS_PROF_SAMPLE);
            launch_sample(c->stream, c->d, c->prec, c->rule, c->b.tab, a);
        }
        c->prop += (uint64_t)c->K;
        {
            PROF(NQS_PROF_THETA);
            launch_theta(c->stream, c->d, c->prec, c->b.tab, c->b.chains, c->C, c->b.tch, nullptr,
                         0);
        }
    }
    return last_launch(c);
}

int nqs_load_samples(nqs_ctx* c, const int8_t* samples, int64_t n_samples) {
    int st = need_bound(c);
    if (st) return st;
    if (!samples || n_samples != c->Ns)
        return fail(c, NQS_EINVAL, "n_samples must equal n_chains * samples_per_chain");
    HIPCHK(c, hipMemcpyAsync(c->b.samples, samples, (size_t)c->Ns * c->N, hipMemcpyDeviceToDevice,
                             c->stream));
    if (c->cplx)
        launch_h_theta(c->stream, c->N, c->M, c->b.hp, c->b.samples, c->Ns, c->b.htsm, nullptr, 0);
    else
        launch_theta(c->stream, c->d, c->prec, c->b.tab, c->b.samples, (int)c->Ns, c->b.tsm,
                     nullptr, 0);
    c->have_samples = true;
    c->have_grad = false;
    return last_launch(c);
}

int nqs_local_energy(nqs_ctx* c, const int8_t* s, int64_t n, double* eloc_out) {
    int st = need_bound(c);
    if (st) return st;
    if (n < 0 || (n > 0 && (!s || !eloc_out))) return fail(c, NQS_EINVAL, "bad batch");
    if (c->cplx) {  // complex energies: (real, imaginary) pairs
        for (int64_t k0 = 0; k0 < n; k0 += c->Bx) {
            const long m = (long)((n - k0) < c->Bx ? (n - k0) : c->Bx);
            const int8_t* sk = s + (size_t)k0 * c->N;
            launch_h_theta(c->stream, c->N, c->M, c->b.hp, sk, m, c->b.htx, nullptr, 0);
            launch_h_eloc(c->stream, c->N, c->M, c->b.hT, c->b.hK, ham_dev(c), sk, c->b.htx, m,
                          (double2*)eloc_out + k0);
        }
        return last_launch(c);
    }
    for (int64_t k0 = 0; k0 < n; k0 += c->Bx) {
        const long m = (long)((n - k0) < c->Bx ? (n - k0) : c->Bx);
        const int8_t* sk = s + (size_t)k0 * c->N;
        launch_theta(c->stream, c->d, c->prec, c->b.tab, sk, (int)m, c->b.tx, nullptr, 0);
        launch_eloc(c->stream, c->d, c->prec, c->b.tab, ham_dev(c), sk, c->b.tx, m, eloc_out + k0,
                    c->lds_limit);
    }
    return last_launch(c);
}

int nqs_local_energy_noalloc(nqs_ctx* c, const int8_t* s, int64_t n, double* eloc_out) {
    int st = need_bound(c);
    if (st) return st;
    if (n < 0 || (n > 0 && (!s || !eloc_out))) return fail(c, NQS_EINVAL, "bad batch");
    if (c->cplx) return fail(c, NQS_EINVAL, "complex models are not supported here");
    const size_t need = esize(c->prec) * (size_t)n * (size_t)c->d.Mw;
    if (need > kNoallocScratchBytes) {
        char msg[160];
        snprintf(msg, sizeof msg,
                 "batch needs %zu bytes of static scratch, more than its %zu bytes; split it",
                 need, kNoallocScratchBytes);
        return fail(c, NQS_EINVAL, msg);
    }
    if (n == 0) return NQS_OK;
    // the same two kernels as nqs_local_energy, over the whole batch at once
    // (each sample's result does not depend on how the batch is cut)
    launch_theta(c->stream, c->d, c->prec, c->b.tab, s, (int)n, c->scratch_dev, nullptr, 0);
    launch_eloc(c->stream, c->d, c->prec, c->b.tab, ham_dev(c), s, c->scratch_dev, (long)n,
                eloc_out, c->lds_limit);
    return last_launch(c);
}

int nqs_log_psi(nqs_ctx* c, const int8_t* s, int64_t n, void* out) {
    int st = need_bound(c);
    if (st) return st;
    if (n < 0 || (n > 0 && (!s || !out))) return fail(c, NQS_EINVAL, "bad batch");
    if (c->cplx) launch_h_log_psi(c->stream, c->N, c->M, c->b.hp, s, n, (double2*)out);
    else launch_log_psi(c->stream, c->d, c->prec, c->b.Pm, c->b.tab, s, n, out);
    return last_launch(c);
}

int nqs_log_psi_vjp(nqs_ctx* c, const int8_t* s, int64_t n, const void* g, void* grad_out) {
    int st = need_bound(c);
    if (st) return st;
    if (n < 0 || (n > 0 && (!s || !g)) || !grad_out) return fail(c, NQS_EINVAL, "bad batch");
    if (c->cplx || c->symm)
        return fail(c, NQS_EINVAL, "complex and symmetric models are not supported here");
    const int PV = c->d.Ma * c->d.Na;
    launch_zero(c->stream, c->b.gacc, 8 * (size_t)PV);
    for (int64_t k0 = 0; k0 < n; k0 += c->Bx) {
        const long m = (long)((n - k0) < c->Bx ? (n - k0) : c->Bx);
        const int8_t* sk = s + (size_t)k0 * c->N;
        launch_theta(c->stream, c->d, c->prec, c->b.tab, sk, (int)m, c->b.tx, nullptr, 0);
        if (c->prec == 0)
            HIPCHK(c, hipMemcpyAsync(c->b.vvec, (const double*)g + k0, 8 * (size_t)m,
                                     hipMemcpyDeviceToDevice, c->stream));
        else
            k_f32_to_f64<<<(unsigned)((m + 255) / 256), 256, 0, c->stream>>>((const float*)g + k0,
                                                                             c->b.vvec, m);
        launch_outer(c->stream, c->d, c->prec, sk, c->b.tx, m, c->b.vvec, 1, c->b.part, c->chunk,
                     c->b.sc);
        launch_reduce_outer(c->stream, c->d, c->prec, c->b.part, outer_ksplit(m, c->chunk),
                            nullptr, 0.0, c->b.Ap, c->b.dpart, c->b.sc, 1);
        launch_axpy_update(c->stream, PV, c->b.gacc, c->b.Ap, -1.0, c->b.sc);
    }
    if (c->prec == 0) {
        launch_pack(c->stream, c->d, c->b.gacc, (double*)grad_out, (int)c->P);
    } else {
        launch_pack(c->stream, c->d, c->b.gacc, c->b.tmpv, (int)c->P);
        k_f64_to_f32<<<(unsigned)((c->P + 255) / 256), 256, 0, c->stream>>>(c->b.tmpv,
                                                                           (float*)grad_out,
                                                                           (long)c->P);
    }
    return last_launch(c);
}

int nqs_jacobian(nqs_ctx* c, const int8_t* s, int64_t n, void* O_out, int center) {
    int st = need_bound(c);
    if (st) return st;
    if (n < 1 || !s || !O_out) return fail(c, NQS_EINVAL, "bad batch");
    if (c->cplx) {  // complex O [n][P], (real, imaginary) pairs
        if (center) return fail(c, NQS_EINVAL, "complex models: uncentred Jacobian only");
        for (int64_t k0 = 0; k0 < n; k0 += c->Bx) {
            const long m = (long)((n - k0) < c->Bx ? (n - k0) : c->Bx);
            const int8_t* sk = s + (size_t)k0 * c->N;
            launch_h_theta(c->stream, c->N, c->M, c->b.hp, sk, m, c->b.htx, nullptr, 0);
            launch_h_jacobian(c->stream, c->N, c->M, sk, c->b.htx, m, (int)c->P,
                              (double2*)O_out + (size_t)k0 * c->P);
        }
        return last_launch(c);
    }
    if (c->symm) {  // FP64 O [n][P_sym]
        for (int64_t k0 = 0; k0 < n; k0 += c->Bx) {
            const long m = (long)((n - k0) < c->Bx ? (n - k0) : c->Bx);
            const int8_t* sk = s + (size_t)k0 * c->N;
            launch_theta(c->stream, c->d, c->prec, c->b.tab, sk, (int)m, c->b.tx, nullptr, 0);
            launch_symm_jacobian(c->stream, c->prec, c->N, c->G, c->alpha, c->vb, c->hb, c->d.Mw,
                                 c->b.perms, sk, c->b.tx, m, c->Psym,
                                 (double*)O_out + (size_t)k0 * c->Psym);
        }
        if (center) {
            if (n > 65535) return fail(c, NQS_EINVAL, "centring supports at most 65535 rows");
            launch_center_cols(c->stream, 0, O_out, n, c->Psym, c->Psym, c->b.tmpv, nullptr, 0,
                               false);
        }
        return last_launch(c);
    }
    const size_t es = esize(c->prec);
    for (int64_t k0 = 0; k0 < n; k0 += c->Bx) {
        const long m = (long)((n - k0) < c->Bx ? (n - k0) : c->Bx);
        const int8_t* sk = s + (size_t)k0 * c->N;
        launch_theta(c->stream, c->d, c->prec, c->b.tab, sk, (int)m, c->b.tx, nullptr, 0);
        launch_jacobian(c->stream, c->d, c->prec, sk, c->b.tx, m,
                        (char*)O_out + es * (size_t)k0 * c->P, (int)c->P, (long)c->P);
    }
    if (center) {
        if (n > 65535) return fail(c, NQS_EINVAL, "centring supports at most 65535 rows");
        launch_center_cols(c->stream, c->prec, O_out, n, (long)c->P, (int)c->P, c->b.tmpv,
                           nullptr, 0, false);
    }
    return last_launch(c);
}

int nqs_expect_and_grad(nqs_ctx* c, nqs_stats* E, double* grad) {
    int st = need_bound(c);
    if (st) return st;
    if (!c->have_samples) return fail(c, NQS_ESTATE, "no samples: call nqs_sample first");
    st = set_device(c);
    if (st) return st;
    if (c->cplx) {
        h_issue_energy_grad(c);
        if (grad) launch_h_join(c->stream, (int)c->P, c->b.fp, (double2*)grad);
    } else {
        issue_energy_grad(c);
        if (c->symm) {  // the plain force, summed over the group
            launch_symm_tie(c->stream, c->N, c->G, c->alpha, c->vb, c->hb, c->d.Na, c->b.perms,
                            c->b.grad, c->b.fp);
            if (grad)
                HIPCHK(c, hipMemcpyAsync(grad, c->b.fp, 8 * (size_t)c->Psym,
                                         hipMemcpyDeviceToDevice, c->stream));
        } else if (grad) {
            launch_pack(c->stream, c->d, c->b.grad, grad, (int)c->P);
        }
    }
    st = last_launch(c);
    if (st) return st;
    if (E) return read_stats(c, E);
    return NQS_OK;
}

// Checks before an SR solve.
static int sr_check(nqs_ctx* c, nqs_qgt kind, double diag_shift, double lr, double tol) {
    int st = need_bound(c);
    if (st) return st;
    if (!c->have_grad) return fail(c, NQS_ESTATE, "no gradient: call nqs_expect_and_grad first");
    if (kind == NQS_QGT_JACOBIAN_DENSE && c->qgt != NQS_QGT_JACOBIAN_DENSE)
        return fail(c, NQS_ESTATE, "dense QGT buffers not in the workspace (nqs_set_qgt)");
    if (c->symm && kind != NQS_QGT_JACOBIAN_DENSE)
        return fail(c, NQS_EINVAL, "symmetric models take the dense QGT");
    if (!(diag_shift >= 0) || !std::isfinite(lr) || !(tol >= 0))
        return fail(c, NQS_EINVAL, "bad solver settings");
    return set_device(c);
}

// The SR solve and update, issued; the CG scalars are not read back here.
static int sr_update_issue(nqs_ctx* c, nqs_qgt kind, double diag_shift, double lr, double tol,
                           int maxiter, double* delta_out) {
    int st = sr_check(c, kind, diag_shift, lr, tol);
    if (st) return st;
    if (c->cplx) {  // G delta = f (complex holomorphic SR), p <- p - lr delta
        st = h_issue_solve(c, diag_shift, tol, maxiter);
        if (st) return st;
        if (delta_out) launch_h_join(c->stream, (int)c->P, c->b.xp, (double2*)delta_out);
        {
            PROF(NQS_PROF_UPDATE);
            launch_h_axpy(c->stream, (int)c->P, c->b.hp, -lr, 0.0, c->b.xp, 0.0, 0.0, nullptr,
                          c->b.hp);
            h_params_changed(c);
        }
        return last_launch(c);
    }
    if (c->symm) {  // (S + eps I) delta = f over the symmetric parameters
        st = s_issue_solve(c, diag_shift, tol, maxiter);
        if (st) return st;
        if (delta_out)
            HIPCHK(c, hipMemcpyAsync(delta_out, c->b.xp, 8 * (size_t)c->Psym,
                                     hipMemcpyDeviceToDevice, c->stream));
        {
            PROF(NQS_PROF_UPDATE);
            launch_axpy_update(c->stream, c->Psym, c->b.psym, c->b.xp, lr, c->b.sc);
            s_params_changed(c);
        }
        return last_launch(c);
    }
    const int mi = default_maxiter(c, maxiter);
    if (kind == NQS_QGT_JACOBIAN_DENSE) issue_dense_setup(c, tol, mi, diag_shift);
    else issue_cg_init(c, tol, mi, diag_shift);
    if (kind == NQS_QGT_JACOBIAN_DENSE && c->dsolver == NQS_SOLVER_CHOLESKY) {
        if (c->prec != 0) return fail(c, NQS_EINVAL, "the Cholesky solve takes the FP64 dense QGT");
        PROF(NQS_PROF_CGVEC);
        launch_chol_solve(c->stream, (double*)c->b.G, (int)c->P, c->Pld, diag_shift, c->b.fp,
                          c->b.xp, c->b.cbad, c->b.cinv, c->b.rp, c->b.sc);
        st = NQS_OK;
    } else {
        st = run_cg(c, kind, diag_shift, mi);
    }
    if (st) return st;
    issue_finish_solve(c, kind);
    if (delta_out) launch_pack(c->stream, c->d, c->b.x, delta_out, (int)c->P);
    issue_update(c, lr);
    return last_launch(c);
}

int nqs_sr_update(nqs_ctx* c, nqs_qgt kind, double diag_shift, double lr, double tol, int maxiter,
                  double* delta_out, nqs_sr_info* info) {
    int st = sr_update_issue(c, kind, diag_shift, lr, tol, maxiter, delta_out);
    if (st) return st;
    st = sync_scalars(c);
    if (st) return st;
    return sr_status(c, info);
}

int nqs_vmc_step(nqs_ctx* c, const nqs_step_cfg* cfg, nqs_step_report* rep) {
    if (!c) return NQS_EINVAL;
    if (!cfg || !rep) return fail(c, NQS_EINVAL, "null settings or report");
    if (c->step_phase) return fail(c, NQS_ESTATE, "a step begun by nqs_step_begin is in flight");
    std::memset(rep, 0, sizeof(*rep));
    int st = nqs_sample(c, 0, nullptr, nullptr, nullptr);
    if (!st) st = nqs_expect_and_grad(c, nullptr, nullptr);
    if (!st) st = sr_update_issue(c, cfg->qgt, cfg->diag_shift, cfg->lr, cfg->cg_tol,
                                  cfg->cg_maxiter, nullptr);
    // the CG scalars, accept counters and energy statistics come back together
    // (one wait for the device)
    if (!st) st = enqueue_scalars(c);
    if (!st) st = enqueue_acceptance(c);
    if (!st) st = enqueue_stats(c);
    if (!st) {
        if (hipStreamSynchronize(c->stream) != hipSuccess)
            st = fail(c, NQS_EDEVICE, "stream synchronise");
    }
    if (!st) st = sr_status(c, &rep->sr);
    if (st == NQS_OK || st == NQS_ENOTCONV) {
        int s2 = take_acceptance(c);
        if (!s2) s2 = take_stats(c, &rep->energy);
        if (s2) st = s2;
    }
    rep->status = st;
    return st;
}

int nqs_tdvp_step(nqs_ctx* c, const nqs_tdvp_cfg* cfg, nqs_tdvp_report* rep) {
    int st = need_bound(c);
    if (st) return st;
    if (!cfg || !rep) return fail(c, NQS_EINVAL, "null settings or report");
    if (!c->cplx) return fail(c, NQS_EINVAL, "TDVP needs a complex (NQS_C128) model");
    if (c->step_phase) return fail(c, NQS_ESTATE, "a step begun by nqs_step_begin is in flight");
    if ((cfg->scheme != NQS_RK_EULER && cfg->scheme != NQS_RK_HEUN) || !std::isfinite(cfg->dt) ||
        !std::isfinite(cfg->gamma_re) || !std::isfinite(cfg->gamma_im) ||
        !(cfg->diag_shift >= 0) || !(cfg->cg_tol >= 0))
        return fail(c, NQS_EINVAL, "bad TDVP settings");
    st = set_device(c);
    if (st) return st;
    std::memset(rep, 0, sizeof(*rep));
    rep->stages = cfg->scheme == NQS_RK_HEUN ? 2 : 1;
    const int P = (int)c->P;
    const double gr = cfg->gamma_re * cfg->dt, gi = cfg->gamma_im * cfg->dt;
    HIPCHK(c, hipMemcpyAsync(c->b.hp0, c->b.hp, 16 * c->P, hipMemcpyDeviceToDevice, c->stream));
    int worst = NQS_OK;
    for (int l = 0; l < rep->stages; ++l) {
        // one evaluation of the equation of motion: x = (G + eps I)^-1 f
        h_issue_sample(c, 0, 1, nullptr);
        h_issue_energy_grad(c);
        st = h_issue_solve(c, cfg->diag_shift, cfg->cg_tol, cfg->cg_maxiter);
        if (!st) st = enqueue_scalars(c);
        if (!st) st = enqueue_acceptance(c);
        if (!st) st = enqueue_stats(c);
        if (!st && hipStreamSynchronize(c->stream) != hipSuccess)
            st = fail(c, NQS_EDEVICE, "stream synchronise");
        if (st) break;
        st = sr_status(c, &rep->solve[l]);
        if (st != NQS_OK && st != NQS_ENOTCONV) break;
        if (st) worst = st;
        take_acceptance(c);
        st = take_stats(c, &rep->energy[l]);
        if (st) break;
        rep->energy_im[l] = c->h_stats[3];
        // theta_dot = gamma x; Euler / Heun's predictor: theta0 + dt gamma x1;
        // Heun's corrector: theta0 + dt gamma (x1 + x2) / 2
        {
            PROF(NQS_PROF_UPDATE);
            if (l == 0) {
                launch_h_axpy(c->stream, P, c->b.hp0, gr, gi, c->b.xp, 0.0, 0.0, nullptr, c->b.hp);
                if (rep->stages == 2)
                    HIPCHK(c, hipMemcpyAsync(c->b.hk1, c->b.xp, 8 * (size_t)c->Pd,
                                             hipMemcpyDeviceToDevice, c->stream));
            } else {
                launch_h_axpy(c->stream, P, c->b.hp0, 0.5 * gr, 0.5 * gi, c->b.hk1, 0.5 * gr,
                              0.5 * gi, c->b.xp, c->b.hp);
            }
            h_params_changed(c);
        }
        st = last_launch(c);
        if (st) break;
    }
    if (!st) st = worst;
    rep->status = st;
    return st;
}

int nqs_batch_step(nqs_ctx* const* ctxs, int n, const nqs_step_cfg* cfgs, nqs_step_report* reps) {
    if (!ctxs || n < 0 || (n > 0 && (!cfgs || !reps))) return NQS_EINVAL;
    std::vector<int> st(n, NQS_OK), mi(n, 0), active(n, 1);
    for (int k = 0; k < n; ++k) {
        std::memset(&reps[k], 0, sizeof(nqs_step_report));
        nqs_ctx* c = ctxs[k];
        st[k] = need_bound(c);
        if (!st[k] && c->step_phase)
            st[k] = fail(c, NQS_ESTATE, "a step begun by nqs_step_begin is in flight");
        if (!st[k] && cfgs[k].qgt == NQS_QGT_JACOBIAN_DENSE && c->qgt != NQS_QGT_JACOBIAN_DENSE)
            st[k] = fail(c, NQS_ESTATE, "dense QGT buffers not in the workspace");
        if (!st[k] && (c->cplx || c->symm))
            st[k] = fail(c, NQS_EINVAL, "complex and symmetric models step one at a time");
        if (!st[k] && cfgs[k].qgt == NQS_QGT_JACOBIAN_DENSE && c->dsolver == NQS_SOLVER_CHOLESKY)
            st[k] = fail(c, NQS_EINVAL, "the Cholesky solve steps one at a time");
        if (!st[k]) st[k] = set_device(c);
    }
    // contexts whose CG iterations may run grouped: small on-the-fly BF16-form
    // contexts on one device (grouping on, no CG kernel class timed), at least two
    std::vector<char> cand(n, 0);
    int gdev = -1;
    {
        int nc = 0;
        for (int k = 0; k < n; ++k) {
            const nqs_ctx* c = ctxs[k];
            if (st[k] || !c->grouping || c->prec == 0 || cfgs[k].qgt != NQS_QGT_ONTHEFLY ||
                (c->prof_mask & CG_CLASSES) || !group_small(c))
                continue;
            if (gdev < 0) gdev = c->device;
            if (c->device == gdev) {
                cand[k] = 1;
                ++nc;
            }
        }
        if (nc < 2) std::fill(cand.begin(), cand.end(), 0);
    }
    // sampling, energies and gradients for every context, then CG init: the
    // grouping candidates first, each recording (flag_ev[0]) when its set-up is
    // done, so that their grouped CG can start while the others still sample
    for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < n; ++k) {
            if (st[k] || (cand[k] != 0) != (pass == 0)) continue;
            nqs_ctx* c = ctxs[k];
            issue_sample(c, 0, nullptr);
            issue_energy_grad(c);
            mi[k] = default_maxiter(c, cfgs[k].cg_maxiter);
            if (cfgs[k].qgt == NQS_QGT_JACOBIAN_DENSE)
                issue_dense_setup(c, cfgs[k].cg_tol, mi[k], cfgs[k].diag_shift);
            else issue_cg_init(c, cfgs[k].cg_tol, mi[k], cfgs[k].diag_shift);
            st[k] = last_launch(c);
            if (!st[k] && cand[k]) {
                const hipError_t e = hipEventRecord(c->flag_ev[0], c->stream);
                if (e != hipSuccess)
                    st[k] = fail(c, NQS_EDEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e));
            }
        }
    // CG on every context side by side: each keeps a batch of iterations queued
    // (two when it runs alone; graph replays where the context allows them) and
    // its stop flag is read as soon as a batch has finished; the host blocks
    // only when no context has a finished batch to read
    std::vector<CgRun> run(n);
    for (int k = 0; k < n; ++k) {
        if (st[k]) continue;
        run[k].init(ctxs[k], cfgs[k].qgt, cfgs[k].diag_shift, mi[k]);
        if (run[k].limit <= 0) active[k] = 0;
    }
    // the candidates that are still fine run their iterations in grouped
    // launches, up to CG_GROUP_MAX per group (at least two); every other context
    // runs its own
    std::vector<CgGroup> groups;
    std::vector<int> gdone;
    std::unique_lock<std::mutex> glock;
    {
        std::vector<int> gk;
        for (int k = 0; k < n; ++k)
            if (cand[k] && !st[k] && active[k]) gk.push_back(k);
        if (gk.size() >= 2) {
            GroupPool& pool = group_pool(gdev);
            glock = std::unique_lock<std::mutex>(pool.m);
            const hipError_t e = hipSetDevice(gdev);
            for (size_t i0 = 0; e == hipSuccess && i0 + 1 < gk.size(); i0 += CG_GROUP_MAX) {
                const size_t i1 = std::min(gk.size(), i0 + (size_t)CG_GROUP_MAX);
                if (i1 - i0 < 2) break;  // (a lone remainder runs its own)
                CgGroup g;
                g.s = group_slot(pool, groups.size(), g.err);
                if (!g.s) break;  // (the remaining contexts run their own)
                int lim = 0;
                for (size_t i = i0; i < i1; ++i) {
                    g.members.push_back(ctxs[gk[i]]);
                    lim = std::max(lim, run[gk[i]].limit);
                    active[gk[i]] = 0;  // driven by the group
                }
                const bool started = g.start(lim);
                if (!started)
                    for (size_t i = i0; i < i1; ++i) st[gk[i]] = fail(ctxs[gk[i]], NQS_EDEVICE, g.err);
                groups.push_back(std::move(g));
                gdone.push_back(started ? 0 : 1);
            }
        }
    }
    auto group_failed = [&](size_t q) {
        for (nqs_ctx* c : groups[q].all)
            for (int k = 0; k < n; ++k)
                if (ctxs[k] == c) st[k] = fail(c, NQS_EDEVICE, groups[q].err);
        gdone[q] = 1;
    };
    bool any = true;
    while (any) {
        any = false;
        bool progress_any = false;
        int wait_on = -1, wait_group = -1;
        for (int k = 0; k < n; ++k) {
            if (st[k] || !active[k]) continue;
            st[k] = run[k].top_up(n > 1 ? 1 : 2);
        }
        for (size_t q = 0; q < groups.size(); ++q)
            if (!gdone[q] && !groups[q].top_up(2)) group_failed(q);
        for (int k = 0; k < n; ++k) {
            if (st[k] || !active[k]) continue;
            bool progress = false;
            st[k] = run[k].poll(false, progress);
            progress_any = progress_any || progress;
            if (st[k] || run[k].finished()) {
                active[k] = 0;
                continue;
            }
            any = true;
            if (wait_on < 0) wait_on = k;
        }
        for (size_t q = 0; q < groups.size(); ++q) {
            if (gdone[q]) continue;
            bool progress = false;
            if (!groups[q].poll(false, progress)) {
                group_failed(q);
                continue;
            }
            progress_any = progress_any || progress;
            if (groups[q].finished()) {
                gdone[q] = 1;
                continue;
            }
            any = true;
            if (wait_group < 0) wait_group = (int)q;
        }
        if (any && !progress_any && wait_on >= 0) {
            bool progress = false;
            st[wait_on] = run[wait_on].poll(true, progress);
            if (st[wait_on] || run[wait_on].finished()) active[wait_on] = 0;
        } else if (any && !progress_any && wait_group >= 0) {
            bool progress = false;
            CgGroup& g = groups[wait_group];
            if (!g.poll(true, progress)) group_failed(wait_group);
            else if (g.finished()) gdone[wait_group] = 1;
        }
    }
    // the members' streams wait for their group's iterations
    for (size_t q = 0; q < groups.size(); ++q)
        if (!groups[q].finish()) group_failed(q);
    for (int k = 0; k < n; ++k) {
        if (st[k]) continue;
        nqs_ctx* c = ctxs[k];
        issue_finish_solve(c, cfgs[k].qgt);
        issue_update(c, cfgs[k].lr);
        st[k] = last_launch(c);
    }
    int first = NQS_OK;
    for (int k = 0; k < n; ++k) {
        nqs_ctx* c = ctxs[k];
        if (!st[k]) st[k] = sync_scalars(c);
        if (!st[k]) st[k] = sr_status(c, &reps[k].sr);
        if (st[k] == NQS_OK || st[k] == NQS_ENOTCONV) {
            int s2 = read_acceptance(c);
            if (!s2) s2 = read_stats(c, &reps[k].energy);
            if (s2) st[k] = s2;
        }
        reps[k].status = st[k];
        if (st[k] && !first) first = st[k];
    }
    return first;
}

// ---- asynchronous steps ---------------------------------------------------
// Ends the step in flight on c (after an error: its kernels may still be queued
// on the stream, which later calls wait behind).
static void step_end(nqs_ctx* c) {
    c->step_phase = 0;
    delete c->step_run;
    c->step_run = nullptr;
}

// Advances the step in flight on c by what is ready (with block, waits for the
// next thing it needs).  completed: its results are on the host.
static int step_advance(nqs_ctx* c, bool block, int depth, bool& progress, bool& completed) {
    progress = completed = false;
    if (c->step_phase == 1) {
        CgRun& r = *c->step_run;
        if (!r.finished()) {
            int st = r.top_up(depth);
            if (st) return st;
            st = r.poll(block, progress);
            if (st) return st;
        }
        if (!r.finished()) return NQS_OK;
        issue_finish_solve(c, c->step_cfg.qgt);
        issue_update(c, c->step_cfg.lr);
        int st = last_launch(c);
        if (!st) st = enqueue_scalars(c);
        if (!st) st = enqueue_acceptance(c);
        if (!st) st = enqueue_stats(c);
        if (st) return st;
        HIPCHK(c, hipEventRecord(c->step_ev, c->stream));
        c->step_phase = 2;
        progress = true;
        block = false;  // (the wait, if any, was for the CG flag)
    }
    if (c->step_phase == 2) {
        const hipError_t e = block ? hipEventSynchronize(c->step_ev) : hipEventQuery(c->step_ev);
        if (e == hipErrorNotReady) return NQS_OK;
        HIPCHK(c, e);
        progress = completed = true;
    }
    return NQS_OK;
}

static void step_report(nqs_ctx* c, nqs_step_report* rep) {
    std::memset(rep, 0, sizeof(*rep));
    int st = sr_status(c, &rep->sr);
    if (st == NQS_OK || st == NQS_ENOTCONV) {
        int s2 = take_acceptance(c);
        if (!s2) s2 = take_stats(c, &rep->energy);
        if (s2) st = s2;
    }
    rep->status = st;
}

int nqs_step_begin(nqs_ctx* c, const nqs_step_cfg* cfg) {
    if (!c) return NQS_EINVAL;
    if (!cfg) return fail(c, NQS_EINVAL, "null settings");
    if (c->step_phase) return fail(c, NQS_ESTATE, "a step is already in flight");
    if (c->cplx || c->symm)
        return fail(c, NQS_EINVAL, "complex and symmetric models step one at a time");
    if (cfg->qgt == NQS_QGT_JACOBIAN_DENSE && c->dsolver == NQS_SOLVER_CHOLESKY)
        return fail(c, NQS_EINVAL, "the Cholesky solve steps one at a time");
    int st = nqs_sample(c, 0, nullptr, nullptr, nullptr);
    if (!st) st = nqs_expect_and_grad(c, nullptr, nullptr);
    if (!st) st = sr_check(c, cfg->qgt, cfg->diag_shift, cfg->lr, cfg->cg_tol);
    if (st) return st;
    const int mi = default_maxiter(c, cfg->cg_maxiter);
    if (cfg->qgt == NQS_QGT_JACOBIAN_DENSE) issue_dense_setup(c, cfg->cg_tol, mi, cfg->diag_shift);
    else issue_cg_init(c, cfg->cg_tol, mi, cfg->diag_shift);
    st = last_launch(c);
    if (st) return st;
    c->step_cfg = *cfg;
    c->step_run = new CgRun();
    c->step_run->init(c, cfg->qgt, cfg->diag_shift, mi);
    c->step_phase = 1;
    if (c->step_run->limit > 0) {
        st = c->step_run->issue_batch();
        if (st) {
            step_end(c);
            return st;
        }
    }
    return NQS_OK;
}

int nqs_step_poll(nqs_ctx* const* ctxs, int n, int wait, nqs_step_report* reps,
                  int32_t* completed) {
    if (!ctxs || n < 0 || (n > 0 && (!reps || !completed))) return NQS_EINVAL;
    for (int k = 0; k < n; ++k) completed[k] = 0;
    const int depth = n > 1 ? 1 : 2;
    int first = NQS_OK;
    auto finish = [&](int k, int st) {
        nqs_ctx* c = ctxs[k];
        if (st) {
            std::memset(&reps[k], 0, sizeof(nqs_step_report));
            reps[k].status = st;
        } else {
            step_report(c, &reps[k]);
        }
        step_end(c);
        completed[k] = 1;
        if (reps[k].status && !first) first = reps[k].status;
    };
    for (;;) {
        bool any_done = false, progress_any = false, inflight = false;
        int wait_on = -1;
        for (int k = 0; k < n; ++k) {
            nqs_ctx* c = ctxs[k];
            if (!c || !c->step_phase || completed[k]) continue;
            bool progress = false, done = false;
            const int st = step_advance(c, false, depth, progress, done);
            if (st || done) {
                finish(k, st);
                any_done = true;
                continue;
            }
            inflight = true;
            progress_any = progress_any || progress;
            if (wait_on < 0) wait_on = k;
        }
        if (!wait || any_done || !inflight) break;
        if (!progress_any) {  // nothing ready anywhere: wait for one context
            bool progress = false, done = false;
            const int st = step_advance(ctxs[wait_on], true, depth, progress, done);
            if (st || done) {
                finish(wait_on, st);
                break;
            }
        }
    }
    return first;
}

int nqs_probe_rate(nqs_ctx* c, nqs_probe kind, double* per_second) {
    if (!c || !per_second) return NQS_EINVAL;
    if (kind < NQS_PROBE_FP32_FMA || kind > NQS_PROBE_BF16_MFMA) return fail(c, NQS_EINVAL, "bad probe");
    int st = set_device(c);
    if (st) return st;
    if (!c->scratch_dev || probe_sink_bytes() > kNoallocScratchBytes)
        return fail(c, NQS_EDEVICE, "no static scratch on this device");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    launch_probe(c->stream, (int)kind, c->scratch_dev);  // warm-up
    HIPCHK(c, hipEventRecord(e0, c->stream));
    double work = 0.0;
    for (int r = 0; r < 3; ++r) work += launch_probe(c->stream, (int)kind, c->scratch_dev);
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    st = last_launch(c);
    if (st) return st;
    *per_second = ms > 0.f ? work / (1e-3 * (double)ms) : 0.0;
    return NQS_OK;
}

int nqs_profile_enable(nqs_ctx* c, uint32_t class_mask) {
    if (!c) return NQS_EINVAL;
    int st = set_device(c);
    if (st) return st;
    if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream));
    if (class_mask && c->ev.empty()) {
        const size_t pairs = 16384;
        c->ev.resize(2 * pairs);
        c->ev_class.assign(pairs, 0);
        for (auto& e : c->ev) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    c->prof_mask = class_mask;
    c->ev_used = 0;
    for (auto& k : c->prof_count) k = 0;
    return NQS_OK;
}

int nqs_profile_read(nqs_ctx* c, double* ms, int64_t* launches, int n) {
    if (!c) return NQS_EINVAL;
    if (n < 0 || n > NQS_PROF_CLASSES) return fail(c, NQS_EINVAL, "bad class count");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<double> tot(NQS_PROF_CLASSES, 0.0);
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float t = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&t, c->ev[i], c->ev[i + 1]));
        tot[c->ev_class[i / 2]] += t;
    }
    for (int k = 0; k < n; ++k) {
        if (ms) ms[k] = tot[k];
        if (launches) launches[k] = c->prof_count[k];
    }
    return NQS_OK;
}

int nqs_set_cg_graphs(nqs_ctx* c, int enable) {
    if (!c) return NQS_EINVAL;
    int st = set_device(c);
    if (st) return st;
    if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->graphs = enable != 0;
    return NQS_OK;
}

int nqs_set_cg_grouping(nqs_ctx* c, int enable) {
    if (!c) return NQS_EINVAL;
    c->grouping = enable != 0;
    return NQS_OK;
}

const char* nqs_profile_class_name(int k) {
    static const char* names[NQS_PROF_CLASSES] = {
        "sample", "theta", "eloc", "stats", "qgt_w", "outer", "reduce", "cg_vec",
        "jacobian", "gram", "dense_matvec", "update", "prepare"};
    return (k >= 0 && k < NQS_PROF_CLASSES) ? names[k] : nullptr;
}

}  // extern "C"
