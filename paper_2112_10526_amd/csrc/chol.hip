// Dense direct solve of (A + shift I) x = f for a symmetric positive-definite A
// (paper: solving the SR / TDVP linear system with a dense QGT; the jVMC
// comparison's dense-solver rows): blocked Cholesky A + shift I = L L^T in
// place (the lower triangle of A becomes L; the upper triangle is never read),
// then L y = f and L^T x = y.  Panels of CH_NB = 32 columns:
//   k_chol_panel  factors the shifted diagonal block in LDS and inverts the
//                 factor (one wave, the block's entries spread over the lanes),
//                 multiplies the panel's rows below by the inverse's transpose
//                 (64-row tiles through LDS), keeps the inverse for the backward solve
//                 and carries the forward solve;
//   k_chol_update subtracts the panel's outer product from the trailing lower
//                 triangle on the FP64 matrix cores (64 x 64 tiles);
// L y = f rides on the panels (each panel forms its y_k and takes its part out
// of the right-hand side of the rows below); L^T x = y runs in one workgroup,
// 32 rows per step, each step a product with the stored inverse of its
// diagonal block.  A pivot
// that is not positive (A + shift I not positive definite) sets *bad.
#include "kernels.h"

namespace nqs {

constexpr int CH_NB = 32;
constexpr int CH_ROWS = 64;  // rows below the diagonal block per panel workgroup

__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ A, int n, long ld, int k0,
                                                    double shift, int32_t* __restrict__ bad,
                                                    double* __restrict__ Yout,
                                                    double* __restrict__ rhs,
                                                    double* __restrict__ yout) {
    __shared__ double D[CH_NB][CH_NB + 1];  // the block, then its factor L_kk
    __shared__ double Y[CH_NB][CH_NB + 1];  // L_kk^-1
    __shared__ double yk[CH_NB];            // this block's part of y = L^-1 f
    __shared__ double fk[CH_NB];            // the panel rows' right-hand side
    __shared__ double Lc[CH_NB][CH_NB + 1]; // the factor's columns, Lc[j][i] = L_ij
    const int w = n - k0 < CH_NB ? n - k0 : CH_NB;
    const int tid = threadIdx.x;
    // the diagonal block's lower part, shifted; identity past w; Y = I
    for (int e = tid; e < CH_NB * CH_NB; e += 256) {
        const int i = e / CH_NB, c = e - i * CH_NB;
        double v = 0.0;
        if (c <= i) {
            if (i < w) v = A[(long)(k0 + i) * ld + k0 + c] + (i == c ? shift : 0.0);
            else if (i == c) v = 1.0;
        }
        D[i][c] = v;
        Y[i][c] = i == c ? 1.0 : 0.0;
    }
    if (tid < CH_NB) fk[tid] = tid < w ? rhs[k0 + tid] : 0.0;
    __syncthreads();
    if (tid < 64) {
        // One wave, the block in registers: lane l holds column c = l % 32 at the
        // rows i = 2 m + l / 32 (m < 16).  Factor step j (unrolled): the pivot
        // comes from its owner by readlane, the two lanes holding column j scale
        // it and publish it (Lc, LDS), then every lane reads its rows' and its
        // column's entries of column j and updates its trailing entries.
        const int l = tid, c = l & 31, par = l >> 5;
        double dr[16], y[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            dr[m] = D[2 * m + par][c];
            y[m] = (2 * m + par == c) ? 1.0 : 0.0;
        }
        bool ok = true;
#pragma unroll
        for (int j = 0; j < CH_NB; ++j) {
            const double djj = readlane(dr[j >> 1], j + 32 * (j & 1));
            ok = ok && djj > 0.0 && isfinite(djj);
            const double d = sqrt(djj > 0.0 ? djj : 1.0), rd = 1.0 / d;
            if (c == j) {
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const int i = 2 * m + par;
                    dr[m] = i == j ? d : (i > j ? dr[m] * rd : dr[m]);
                    Lc[j][i] = dr[m];
                }
            }
            __builtin_amdgcn_wave_barrier();
            double lr_[16];
#pragma unroll
            for (int m = 0; m < 16; ++m) lr_[m] = Lc[j][2 * m + par];
            const double lcj = Lc[j][c];
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int i = 2 * m + par;
                if (c > j && i >= c) dr[m] -= lr_[m] * lcj;
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (!ok && blockIdx.x == 0 && l == 0) *bad = 1;
        // Y = L_kk^-1 by row operations on the identity (same layout): step j
        // scales row j by 1 / L_jj, then row i -= L_ij row j for i > j; Y[j][c]
        // comes from the lane holding row j's parity (this lane or l ^ 32)
#pragma unroll
        for (int j = 0; j < CH_NB; ++j) {
            const double rjj = 1.0 / Lc[j][j];
            if (par == (j & 1)) y[j >> 1] *= rjj;
            const double mine = y[j >> 1];
            const double other = __shfl_xor(mine, 32);
            const double yjc = par == (j & 1) ? mine : other;
            double lr_[16];
#pragma unroll
            for (int m = 0; m < 16; ++m) lr_[m] = Lc[j][2 * m + par];
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int i = 2 * m + par;
                if (i > j) y[m] -= lr_[m] * yjc;
            }
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            D[2 * m + par][c] = dr[m];
            Y[2 * m + par][c] = y[m];
        }
    }
    // y_k = L_kk^-1 f_k (f_k as left by the earlier panels; every block forms it,
    // no block writes the rhs rows of this panel)
    if (tid < CH_NB) {
        double y = 0.0;
#pragma unroll
        for (int m = 0; m < CH_NB; ++m) y += Y[tid][m] * fk[m];  // (Y lower; fk zero past w)
        yk[tid] = tid < w ? y : 0.0;
    }
    __syncthreads();
    if (blockIdx.x == 0) {  // the factor into A; the inverse and y_k to the side
        for (int e = tid; e < CH_NB * CH_NB; e += 256) {
            const int i = e / CH_NB, c = e - i * CH_NB;
            if (i < w && c <= i) A[(long)(k0 + i) * ld + k0 + c] = D[i][c];
            Yout[(size_t)(k0 / CH_NB) * CH_NB * CH_NB + e] = Y[i][c];
        }
        if (tid < w) yout[k0 + tid] = yk[tid];
        return;
    }
    // rows below the block, 64 per block: x = a L_kk^-T, x_c = sum_m a_m
    // (L_kk^-1)[c][m], and each row's right-hand side loses x . y_k.  The tile
    // moves through LDS so that its loads and stores are coalesced; thread t
    // computes row t / 4, columns 8 (t % 4) .. + 7.
    __shared__ double T[CH_ROWS][CH_NB + 1];
    const long r0 = (long)k0 + w + (long)(blockIdx.x - 1) * CH_ROWS;
    const int tr = tid >> 2, tc = (tid & 3) * 8;
    const long r = r0 + tr;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        T[tr][tc + q] = (r < n && tc + q < w) ? A[r * ld + k0 + tc + q] : 0.0;
    __syncthreads();
    double xo[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xo[q] = 0.0;
#pragma unroll
    for (int m = 0; m < CH_NB; ++m) {
        const double t = T[tr][m];
#pragma unroll
        for (int q = 0; q < 8; ++q) xo[q] += t * Y[tc + q][m];
    }
    double fr = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) fr += xo[q] * yk[tc + q];
    fr += __shfl_xor(fr, 1);
    fr += __shfl_xor(fr, 2);
    if (r < n) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (tc + q < w) A[r * ld + k0 + tc + q] = xo[q];
        if ((tid & 3) == 0) rhs[r] -= fr;
    }
}

// trailing update T -= X X^T on the lower triangle, T = A[k1:, k1:], X = A[k1:, k0:k1];
// block = a 64 x 64 tile (ti >= tj), wave = a 32 x 32 quarter of 2 x 2 MFMA tiles
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ A, int n, long ld, int k0,
                                                     int k1) {
    const long b = blockIdx.x;
    long ti = (long)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
    while (ti * (ti + 1) / 2 > b) --ti;
    const long tj = b - ti * (ti + 1) / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long ri = k1 + ti * 64 + (wave >> 1) * 32, cj = k1 + tj * 64 + (wave & 1) * 32;
    const int w = k1 - k0;
    v4d acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = v4d{0, 0, 0, 0};
    for (int kk = 0; kk < w; kk += 4) {
        const int k = kk + lk;
        double fa[2], fb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const long rr = ri + a * 16 + lr, cc = cj + a * 16 + lr;
            fa[a] = (rr < n && k < w) ? A[rr * ld + k0 + k] : 0.0;
            fb[a] = (cc < n && k < w) ? A[cc * ld + k0 + k] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[c], acc[a][c], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const long row = ri + a * 16 + acc_row<double>(lk, q), col = cj + c * 16 + lr;
                if (row < n && col <= row) A[row * ld + col] -= acc[a][c][q];
            }
}

// L^T x = y, one workgroup of 1024 threads, a 32-row block per step from the
// last: x_k = Yinv_k^T (y_k - sum_{j>k} L_jk^T x_j), Yinv_k (the inverse of the
// diagonal block, [blocks][32][32]) staged in LDS
__global__ __launch_bounds__(1024) void k_chol_back(const double* __restrict__ L, int n, long ld,
                                                    const double* __restrict__ Yinv,
                                                    const double* __restrict__ y,
                                                    double* __restrict__ x) {
    __shared__ double red[16][CH_NB];
    __shared__ double sv[CH_NB];
    __shared__ double Yk[CH_NB * CH_NB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nblk = (n + CH_NB - 1) / CH_NB;
    for (int kb = nblk - 1; kb >= 0; --kb) {
        const int k0 = kb * CH_NB;
        const int w = n - k0 < CH_NB ? n - k0 : CH_NB;
        Yk[threadIdx.x] = Yinv[(size_t)kb * CH_NB * CH_NB + threadIdx.x];
        // partial sums over j >= k0 + w of L[j][k0 + i] x[j], rows j split over the waves
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        if (lane < w) {
            long j = k0 + w + wave;
            for (; j + 48 < n; j += 64) {  // four independent rows in flight
                a0 += L[j * ld + k0 + lane] * x[j];
                a1 += L[(j + 16) * ld + k0 + lane] * x[j + 16];
                a2 += L[(j + 32) * ld + k0 + lane] * x[j + 32];
                a3 += L[(j + 48) * ld + k0 + lane] * x[j + 48];
            }
            for (; j < n; j += 16) a0 += L[j * ld + k0 + lane] * x[j];
        }
        if (lane < CH_NB) red[wave][lane] = (a0 + a1) + (a2 + a3);
        __syncthreads();
        if (wave == 0 && lane < CH_NB) {
            double t = 0.0;
            for (int v = 0; v < 16; ++v) t += red[v][lane];
            sv[lane] = lane < w ? y[k0 + lane] - t : 0.0;
        }
        __syncthreads();
        if (wave == 0 && lane < w) {  // x_i = sum_m Yinv[m][i] s_m, m >= i
            double xi = 0.0;
            for (int m = lane; m < w; ++m) xi += Yk[m * CH_NB + lane] * sv[m];
            x[k0 + lane] = xi;
        }
        __syncthreads();
    }
}

// CG scalars of a direct solve: no iterations, converged, zero residual (the
// solve is exact up to rounding), bad when a pivot was not positive
__global__ void k_chol_status(const int32_t* __restrict__ bad, CgScalars* sc) {
    if (threadIdx.x) return;
    sc->iters = 0;
    sc->rr = 0.0;
    sc->rr0 = 1.0;
    sc->tol2 = 0.0;
    sc->done = 1;
    sc->bad = *bad ? 1 : 0;
}

// ---------------------------------------------------------------------------
size_t chol_side_bytes(int n) { return (size_t)((n + CH_NB - 1) / CH_NB) * CH_NB * CH_NB * 8; }
__global__ void k_copy_vec(const double* __restrict__ a, double* __restrict__ b, int n) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < n) b[e] = a[e];
}

void launch_chol_solve(hipStream_t st, double* A, int n, long ld, double shift, const double* f,
                       double* x, int32_t* bad, double* Yinv, double* y, CgScalars* sc) {
    launch_zero(st, bad, sizeof(int32_t));
    // x holds the right-hand side as the panels eliminate it (L y = f), y gets y
    k_copy_vec<<<(n + 255) / 256, 256, 0, st>>>(f, x, n);
    for (int k0 = 0; k0 < n; k0 += CH_NB) {
        const int w = n - k0 < CH_NB ? n - k0 : CH_NB;
        const int below = n - k0 - w;
        k_chol_panel<<<1 + (below + CH_ROWS - 1) / CH_ROWS, 256, 0, st>>>(A, n, ld, k0, shift,
                                                                          bad, Yinv, x, y);
        if (below > 0) {
            const long mt = (below + 63) / 64;
            k_chol_update<<<(unsigned)(mt * (mt + 1) / 2), 256, 0, st>>>(A, n, ld, k0, k0 + w);
        }
    }
    k_chol_back<<<1, 1024, 0, st>>>(A, n, ld, Yinv, y, x);
    k_chol_status<<<1, 64, 0, st>>>(bad, sc);
}

}  // namespace nqs
