// Dense direct solve of (A + shift I) x = f for a symmetric positive-definite A
// (paper: solving the SR / TDVP linear system with a dense QGT; the jVMC
// comparison's dense-solver rows): blocked Cholesky A + shift I = L L^T in
// place (the lower triangle of A becomes L; the upper triangle is never read),
// then L y = f and L^T x = y.  Panels of CH_NB = 32 columns:
//   k_chol_panel  factors the shifted diagonal block in LDS (one wave, a row per
//                 lane), inverts the factor (a column per lane) and multiplies
//                 the panel's rows below by its transpose (a row per thread);
//   k_chol_update subtracts the panel's outer product from the trailing lower
//                 triangle on the FP64 matrix cores (64 x 64 tiles);
// the two triangular solves run in one workgroup, 32 rows per step.  A pivot
// that is not positive (A + shift I not positive definite) sets *bad.
#include "kernels.h"

namespace nqs {

constexpr int CH_NB = 32;

__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ A, int n, long ld, int k0,
                                                    double shift, int32_t* __restrict__ bad) {
    __shared__ double D[CH_NB][CH_NB + 1];  // the block, then its factor L_kk
    __shared__ double Y[CH_NB][CH_NB + 1];  // L_kk^-1
    const int w = n - k0 < CH_NB ? n - k0 : CH_NB;
    const int tid = threadIdx.x;
    // the diagonal block's lower part, shifted; identity past w
    for (int e = tid; e < CH_NB * CH_NB; e += 256) {
        const int i = e / CH_NB, c = e - i * CH_NB;
        double v = 0.0;
        if (c <= i) {
            if (i < w) v = A[(long)(k0 + i) * ld + k0 + c] + (i == c ? shift : 0.0);
            else if (i == c) v = 1.0;
        }
        D[i][c] = v;
    }
    __syncthreads();
    if (tid < CH_NB) {
        // one wave, lane i = row i: right-looking factor in LDS (a wave's LDS
        // operations complete in order, so the wave barriers only pin the order)
        const int i = tid;
        bool ok = true;
        for (int j = 0; j < CH_NB; ++j) {
            const double djj = D[j][j];
            ok = ok && djj > 0.0 && isfinite(djj);
            const double d = sqrt(djj > 0.0 ? djj : 1.0);
            __builtin_amdgcn_wave_barrier();
            if (i == j) D[j][j] = d;
            if (i > j) D[i][j] /= d;
            __builtin_amdgcn_wave_barrier();
            if (i > j) {
                const double lij = D[i][j];
                for (int c = j + 1; c <= i; ++c) D[i][c] -= lij * D[c][j];
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (!ok && blockIdx.x == 0 && i == 0) *bad = 1;
        // lane c: column c of L_kk^-1 by forward substitution (lanes independent)
        const int c = tid;
        for (int r = 0; r < CH_NB; ++r) {
            double v = 0.0;
            if (r >= c) {
                double t = r == c ? 1.0 : 0.0;
                for (int m = c; m < r; ++m) t -= D[r][m] * Y[m][c];
                v = t / D[r][r];
            }
            Y[r][c] = v;
        }
    }
    __syncthreads();
    if (blockIdx.x == 0) {
        for (int e = tid; e < CH_NB * CH_NB; e += 256) {
            const int i = e / CH_NB, c = e - i * CH_NB;
            if (i < w && c <= i) A[(long)(k0 + i) * ld + k0 + c] = D[i][c];
        }
        return;
    }
    // rows below the block: x = a L_kk^-T, x_c = sum_m a_m (L_kk^-1)[c][m]
    const long r = (long)k0 + w + (long)(blockIdx.x - 1) * 256 + tid;
    if (r >= n) return;
    double* ar = A + r * ld + k0;
    double av[CH_NB];
#pragma unroll
    for (int m = 0; m < CH_NB; ++m) av[m] = m < w ? ar[m] : 0.0;
    for (int c = 0; c < w; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < CH_NB; ++m) acc += av[m] * Y[c][m];
        ar[c] = acc;
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

// L y = f, then L^T x = y (x may alias f), one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void k_chol_solve(const double* __restrict__ L, int n, long ld,
                                                     const double* f, double* x) {
    __shared__ double red[16][CH_NB];
    __shared__ double sv[CH_NB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // forward
    for (int k0 = 0; k0 < n; k0 += CH_NB) {
        const int w = n - k0 < CH_NB ? n - k0 : CH_NB;
        for (int rr = wave; rr < w; rr += 16) {  // s_r = f_r - sum_{j < k0} L[r][j] y[j]
            const long r = k0 + rr;
            double a = 0.0;
            for (int j = lane; j < k0; j += 64) a += L[r * ld + j] * x[j];
            a = wave_sum(a);
            if (lane == 0) sv[rr] = f[r] - a;
        }
        __syncthreads();
        if (wave == 0) {
            const int i = lane;
            double s = i < w ? sv[i] : 0.0;
            double yi = 0.0;
            for (int c = 0; c < w; ++c) {
                const double yc = readlane(s, c) / L[(long)(k0 + c) * ld + k0 + c];
                if (i == c) yi = yc;
                if (i > c && i < w) s -= L[(long)(k0 + i) * ld + k0 + c] * yc;
            }
            if (i < w) x[k0 + i] = yi;
        }
        __syncthreads();
    }
    // backward
    const int nblk = (n + CH_NB - 1) / CH_NB;
    for (int kb = nblk - 1; kb >= 0; --kb) {
        const int k0 = kb * CH_NB;
        const int w = n - k0 < CH_NB ? n - k0 : CH_NB;
        // partial sums over j >= k0 + w of L[j][k0 + i] x[j], rows j split over the waves
        double a = 0.0;
        if (lane < w)
            for (long j = k0 + w + wave; j < n; j += 16) a += L[j * ld + k0 + lane] * x[j];
        if (lane < CH_NB) red[wave][lane] = a;
        __syncthreads();
        if (wave == 0) {
            const int i = lane;
            double s = 0.0;
            if (i < w) {
                double t = 0.0;
                for (int v = 0; v < 16; ++v) t += red[v][i];
                s = x[k0 + i] - t;
            }
            double xi = 0.0;
            for (int c = w - 1; c >= 0; --c) {
                const double xc = readlane(s, c) / L[(long)(k0 + c) * ld + k0 + c];
                if (i == c) xi = xc;
                if (i < c) s -= L[(long)(k0 + c) * ld + k0 + i] * xc;
            }
            if (i < w) x[k0 + i] = xi;
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
void launch_chol_solve(hipStream_t st, double* A, int n, long ld, double shift, const double* f,
                       double* x, int32_t* bad, CgScalars* sc) {
    launch_zero(st, bad, sizeof(int32_t));
    for (int k0 = 0; k0 < n; k0 += CH_NB) {
        const int w = n - k0 < CH_NB ? n - k0 : CH_NB;
        const int below = n - k0 - w;
        k_chol_panel<<<1 + (below + 255) / 256, 256, 0, st>>>(A, n, ld, k0, shift, bad);
        if (below > 0) {
            const long mt = (below + 63) / 64;
            k_chol_update<<<(unsigned)(mt * (mt + 1) / 2), 256, 0, st>>>(A, n, ld, k0, k0 + w);
        }
    }
    k_chol_solve<<<1, 1024, 0, st>>>(A, n, ld, f, x);
    k_chol_status<<<1, 64, 0, st>>>(bad, sc);
}

}  // namespace nqs
