// Factor readout of a returns stream (Section 5): causal de-meaning of the
// rows (Section 5.1), the low-rank covariance implied by the factors, and
// the k-sized products behind portfolio volatility and the covariance error
// (Section 5.3).  Bases are in the tiled layout of isvd_common.h (uvo).
#pragma once
#include "isvd_common.h"

namespace isvd {

// Expanding mean per column, rows in order (Section 5.1):
// mu_t = mu_{t-1} + (r_t - mu_{t-1}) / t, R_t = r_t - mu_t, in FP64.  One
// thread per column; out may alias r (each element is read, then written,
// by the same thread).
template <typename T>
__global__ void __launch_bounds__(256) k_causal_center(const T* r, T* out, int64_t rows, int64_t n, double* mu,
                                                       int64_t t0) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    double m = t0 > 0 ? mu[j] : 0.0;
    for (int64_t q = 0; q < rows; ++q) {
        const double t = (double)(t0 + q + 1);
        const double x = (double)r[q * n + j];
        m = m + (x - m) / t;
        out[q * n + j] = (T)(x - m);
    }
    mu[j] = m;
}

constexpr int kCovTile = 64;   // output tile edge; 16 x 16 threads, 4 x 4 entries each
constexpr int kCovChunk = 16;  // columns of V staged per step

// C = V diag(S^2) V^T / (m - 1) (n x n, FP64, ldc) from the stream's
// current tiled basis: k, ld, the current buffer and m come from the device
// header, so the launch needs no host round trip; n is the host's view
// (equal to the header's once the stream's queued updates have run).
// Block (bx, by) computes a 64 x 64 tile; thread (ty, tx) holds entries
// (ty + 16 a, tx + 16 b), a, b < 4, in registers.  V's row panels are staged
// 16 columns at a time in LDS as FP64 (columns k.. read as zero).  Entry
// (i, j) adds (V_ic V_jc) S_c^2 in order of c, so C is exactly symmetric.
template <typename T>
__global__ void __launch_bounds__(256) k_lowrank_cov(const DevHeader* __restrict__ hdr, const T* V0, const T* V1,
                                                     const double* __restrict__ S, int64_t n, double* __restrict__ C,
                                                     int64_t ldc) {
    const int k = hdr->k, ld = hdr->ld;
    const T* __restrict__ V = hdr->cur ? V1 : V0;
    const double scale = 1.0 / (double)(hdr->m - 1);
    __shared__ double a[kCovChunk][kCovTile + 1];
    __shared__ double b[kCovChunk][kCovTile + 1];
    __shared__ double s2[kCovChunk];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t i0 = (int64_t)blockIdx.y * kCovTile, j0 = (int64_t)blockIdx.x * kCovTile;
    double acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
    for (int c0 = 0; c0 < k; c0 += kCovChunk) {
        // 64 rows x 16 columns of each panel: thread t loads rows t / 16 + 16 p, column t % 16
        const int cc = threadIdx.x % kCovChunk, rr = threadIdx.x / kCovChunk;
        const int c = c0 + cc;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int row = rr + 16 * p;
            a[cc][row] = (c < k && i0 + row < n) ? (double)V[uvo(i0 + row, c, ld)] : 0.0;
            b[cc][row] = (c < k && j0 + row < n) ? (double)V[uvo(j0 + row, c, ld)] : 0.0;
        }
        if (threadIdx.x < kCovChunk) s2[threadIdx.x] = c0 + (int)threadIdx.x < k ? S[c0 + threadIdx.x] * S[c0 + threadIdx.x] : 0.0;
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < kCovChunk; ++q) {
            double x[4], y[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                x[p] = a[q][ty + 16 * p];
                y[p] = b[q][tx + 16 * p];
            }
            const double sq = s2[q];
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[p][r] += (x[p] * y[r]) * sq;
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int64_t i = i0 + ty + 16 * p;
        if (i >= n) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = j0 + tx + 16 * r;
            if (j < n) C[i * ldc + j] = acc[p][r] * scale;
        }
    }
}

// y_c = sum_r V[r][c] w_r: one block per column c; thread t adds rows
// t, t + 256, ... in order, then a fixed-order tree over the threads.
template <typename T>
__global__ void __launch_bounds__(256) k_vt_w(const T* __restrict__ V, int ld, int64_t n, const double* __restrict__ w,
                                              double* __restrict__ y) {
    __shared__ double red[256];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += 256) acc += (double)V[uvo(r, c, ld)] * w[r];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) y[c] = red[0];
}

// out[i * kb + j] = sum_r A[r][i] B[r][j] (A: n x ka, B: n x kb, tiled bases):
// one block per i, one thread per j, rows in order.
template <typename TA, typename TB>
__global__ void __launch_bounds__(128) k_cross(const TA* __restrict__ A, int lda, const TB* __restrict__ B, int ldb,
                                               int64_t n, int kb, double* __restrict__ out) {
    const int i = blockIdx.x, j = threadIdx.x;
    if (j >= kb) return;
    double acc = 0.0;
    for (int64_t r = 0; r < n; ++r) acc += (double)A[uvo(r, i, lda)] * (double)B[uvo(r, j, ldb)];
    out[(size_t)i * kb + j] = acc;
}

}  // namespace isvd
