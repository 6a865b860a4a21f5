// Refresh kernels, Gram form: TruncatedSVD(A_t, k) (Algorithm 1 init and
// refresh, Section 2.4.1) for streams of at most kGcfMaxN columns, iterated
// until the leading k Ritz pairs have converged.
//
// The truncated SVD of A is the leading part of the eigen-decomposition of
// its Gram matrix G = A^T A (right vectors, sigma^2).  G is formed once per
// refresh from A on the FP64 matrix cores (products of FP32 or FP64 entries
// are exact in FP64 and accumulate in FP64), and the subspace iteration then
// runs on the n x n matrix G instead of the m x n matrix A:
//
//   X (n x b) orthonormal start (V_t and pseudo-random columns)
//   loop:
//     Rayleigh-Ritz on the active block:  W = G_d X,  H = X^T W,
//       H = R^T R (Cholesky),  R = . Sigma P^T (one-sided Jacobi),
//       X <- X P,  W <- W P,  theta = sigma^2,  res_j = ||W_j - theta_j X_j||
//     stop when the leading k pairs have res_j <= tol theta_1, or when their
//       largest residual stops halving from one round to the next within
//       1e3 tol theta_1 (it has reached rounding level)
//     lock the leading pairs that sit far above the cut (theta_j >= 16
//       theta_cut, the factor directions) once res_j <= max(tol, 1e-14)
//       theta_1, and deflate them out of the operator:
//       G_d <- (I - L L^T) G_d (I - L L^T)   (a symmetric rank-2 update);
//       pairs inside the bulk stay active and keep improving: a pair frozen
//       as soon as it met the tolerance would keep an error of its residual
//       over its (tiny) gap; the active block is refilled with fresh
//       columns to min(b, n - locked), so the locked vectors and the block
//       together can reach past b (k up to 128 with a block of at most 128)
//     Chebyshev filter of degree d on [0, theta_cut] (theta_cut the smallest
//       active Ritz value): Y_{j+1} = (2/e)(G_d - c) Y_j - Y_{j-1},
//       c = e = theta_cut / 2, so the unwanted part of the spectrum stays
//       bounded by 1 while every eigenvalue above theta_cut grows like
//       cosh(d acosh(2 lambda / theta_cut - 1)); d is the largest degree that
//       keeps the growth of the largest active Ritz value below 1e6, so the
//       filtered block stays well conditioned for CholQR2
//     X <- CholQR2(Y - L L^T Y)
//
// Deflating the converged pairs far above the cut is what lets the filter
// run at high degree: the factor directions of a factor-model panel sit
// orders of magnitude above the noise bulk, and left in the operator they
// would swamp the block after one filter step.  The method is Chebyshev-filtered
// subspace iteration (Zhou and Saad 2007) with locking; the stopping rule is
// the Ritz residual, which bounds the eigenvalue error of a Ritz pair of a
// symmetric matrix (|theta - lambda| <= res) and, divided by the spectral
// gap, its angle.  The block of the locked right vectors L and the leading
// remaining active ones then goes through the same final step as the A-form
// refresh: Y = A X, CholQR2, SVD of R, which yields U, Sigma, V with U
// orthonormal to working precision.  G's rounding (relative to sigma_1^2)
// mixes the directions next to the cut, whose gap may be tiny inside a
// noise bulk; the block holds those neighbours, and the Rayleigh-Ritz step
// on A separates them at the accuracy of A.
//
// All G-space blocks are FP64, np = round64(n) rows (rows past n zero) and a
// width w that is a multiple of 16 with zero columns past the active count;
// zero columns pass through every step (the Cholesky drops them, the Jacobi
// gives them zero singular values, sorted last).
#pragma once
#include "isvd_common.h"
#include "isvd_refresh.h"

namespace isvd {

constexpr int kGcfMaxN = 4096;     // widest stream refreshed in Gram form
constexpr int kAtaTile = 128;     // Gram tile edge
constexpr int kAtaStage = 16;     // rows of A per LDS stage of the Gram product
constexpr int kAtaLd = 2 * kAtaTile + 4;   // LDS row stride (doubles) of a stage

__host__ __device__ inline int64_t round64(int64_t v) { return (v + 63) & ~(int64_t)63; }
__host__ __device__ inline int ata_panels(int64_t n) { return (int)((n + kAtaTile - 1) / kAtaTile); }
__host__ __device__ inline int ata_tiles(int64_t n) {
    const int p = ata_panels(n);
    return p * (p + 1) / 2;
}
// tile t of the upper triangle of tiles, row by row
__device__ inline void ata_tile(int t, int np, int* ip, int* jp) {
    int i = 0;
    while (t >= np - i) {
        t -= np - i;
        ++i;
    }
    *ip = i;
    *jp = i + t;
}

// Partial Gram tiles: Gp[chunk][tile][128 x 128] = sum over the rows of the
// chunk of A[r][128 ip + a] A[r][128 jp + c].  grid (tiles, chunks), 256
// threads; a stage of 16 rows of the two 128-column panels is held in LDS
// as FP64 (the next stage prefetched into registers); wave w owns the
// 64 x 64 quadrant (w / 2, w % 2) of the tile, sixteen 16 x 16 FP64 MFMA
// tiles, so each LDS operand read feeds four MFMAs.
// MFMA operands: lane l gives A_op[l % 16][l / 16] = A[r0 + l / 16][128 ip + ...]
// and B_op[l / 16][l % 16] = A[r0 + l / 16][128 jp + ...], so D = A_op B_op is
// a block of the (ip, jp) tile of A^T A.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_ata_mfma(const T* __restrict__ A, int64_t lda, int64_t m,
                                                       int64_t n, int64_t rpc, double* __restrict__ Gp) {
    constexpr int PER = kAtaStage * 2 * kAtaTile / kThreads;   // 16
    __shared__ double sA[kAtaStage][kAtaLd];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int npan = ata_panels(n), ntile = npan * (npan + 1) / 2;
    int ip, jp;
    ata_tile(blockIdx.x, npan, &ip, &jp);
    const int64_t ci = (int64_t)ip * kAtaTile, cj = (int64_t)jp * kAtaTile;
    const int64_t ra = (int64_t)blockIdx.y * rpc;
    const int64_t rb = min(m, ra + rpc);
    T pre[PER];
    auto fetch = [&](int64_t r0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + kThreads * q;
            const int rr = e >> 8, cc = e & 255;
            const int64_t col = cc < kAtaTile ? ci + cc : cj + cc - kAtaTile;
            const int64_t r = r0 + rr;
            pre[q] = (r < rb && col < n) ? A[r * lda + col] : (T)0;
        }
    };
    mm_v4d acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = (mm_v4d){0.0, 0.0, 0.0, 0.0};
    const int oi = (w >> 1) * 64 + (l & 15), oj = kAtaTile + (w & 1) * 64 + (l & 15);
    if (ra < rb) fetch(ra);
    for (int64_t r0 = ra; r0 < rb; r0 += kAtaStage) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + kThreads * q;
            sA[e >> 8][e & 255] = (double)pre[q];
        }
        __syncthreads();
        if (r0 + kAtaStage < rb) fetch(r0 + kAtaStage);
#pragma unroll
        for (int kk = 0; kk < kAtaStage / 4; ++kk) {
            const int rr = 4 * kk + (l >> 4);
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                av[a] = sA[rr][oi + 16 * a];
                bv[a] = sA[rr][oj + 16 * a];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0, 0, 0);
        }
        __syncthreads();
    }
    double* out = Gp + ((int64_t)blockIdx.y * ntile + blockIdx.x) * (kAtaTile * kAtaTile);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = (w >> 1) * 64 + 16 * a + 4 * r + (l >> 4);
                const int col = (w & 1) * 64 + 16 * c + (l & 15);
                out[row * kAtaTile + col] = acc[a][c][r];
            }
}

// G (ldg x ldg, row-major) = sum of the chunk partials in chunk order; an
// element of the lower triangle (and of the lower half of a diagonal tile)
// is read from its mirror, so G is exactly symmetric; rows / columns past n
// are zero.  One thread per element of G.
__global__ void k_ata_sum(const double* __restrict__ Gp, int nchunk, int64_t n, int ldg, double* __restrict__ G) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)ldg * ldg) return;
    int64_t i = e / ldg, j = e % ldg;
    if (i >= n || j >= n) {
        G[e] = 0.0;
        return;
    }
    if (i / kAtaTile > j / kAtaTile || (i / kAtaTile == j / kAtaTile && i > j)) {
        const int64_t t = i;
        i = j;
        j = t;
    }
    constexpr int64_t TT = (int64_t)kAtaTile * kAtaTile;
    const int npan = ata_panels(n), ntile = npan * (npan + 1) / 2;
    const int ip = (int)(i / kAtaTile), jp = (int)(j / kAtaTile);
    // index of tile (ip, jp) in the row-by-row upper triangle
    const int tile = ip * npan - ip * (ip - 1) / 2 + (jp - ip);
    const double* P = Gp + (int64_t)tile * TT + (i % kAtaTile) * kAtaTile + (j % kAtaTile);
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += P[(int64_t)c * ntile * TT];
    G[e] = s;
}

// Out = alpha (G Y1) + beta Y1 + gamma Y0 (Y0 unused when gamma == 0; Out
// may be Y0: each element of Y0 is read by the thread that writes it), all
// FP64; G ldg x ldg symmetric (ldg a multiple of 64, zero past n), Y ldg x w
// with leading dimension ldy (w a multiple of 16).  Block (256 threads)
// computes a 16-row x 32-column tile; its four waves split the inner
// dimension into quarters and their MFMA tiles are added in LDS in wave
// order.  A_op[i][k] = G[k0 + k][i0 + i] (G symmetric: rows of G are read,
// 16 consecutive doubles per lane group), B_op[k][j] = Y1[k0 + k][j0 + j].
__global__ void __launch_bounds__(kThreads) k_symm_cheb(const double* __restrict__ G, int ldg,
                                                        const double* __restrict__ Y1,
                                                        const double* Y0, double* Out,
                                                        int ldy, int w, double alpha, double beta, double gamma) {
    __shared__ double red[4][16][33];
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 32;
    const bool two = j0 + 16 < w;
    const int kq = ldg / 4;   // a multiple of 16
    const int ks = wv * kq, ke = ks + kq;
    mm_v4d acc0 = (mm_v4d){0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    const int lr = l >> 4, lc = l & 15;
    const double* gp = G + (int64_t)(ks + lr) * ldg + i0 + lc;
    const double* yp = Y1 + (int64_t)(ks + lr) * ldy + j0 + lc;
    // kq is a multiple of 16: four MFMA steps per iteration, loads issued first
    const int64_t sg = 4 * (int64_t)ldg, sy = 4 * (int64_t)ldy;
    if (two) {
        for (int k0 = ks; k0 < ke; k0 += 16) {
            double a[4], b0[4], b1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = gp[u * sg];
                b0[u] = yp[u * sy];
                b1[u] = yp[u * sy + 16];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b0[u], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b1[u], acc1, 0, 0, 0);
            }
            gp += 4 * sg;
            yp += 4 * sy;
        }
    } else {
        for (int k0 = ks; k0 < ke; k0 += 16) {
            double a[4], b0[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = gp[u * sg];
                b0[u] = yp[u * sy];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b0[u], acc0, 0, 0, 0);
            gp += 4 * sg;
            yp += 4 * sy;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        red[wv][4 * r + lr][lc] = acc0[r];
        red[wv][4 * r + lr][16 + lc] = acc1[r];
    }
    __syncthreads();
    const int ncol = two ? 32 : 16;
    for (int e = threadIdx.x; e < 16 * ncol; e += kThreads) {
        const int r = e / ncol, c = e % ncol;
        const double s = ((red[0][r][c] + red[1][r][c]) + red[2][r][c]) + red[3][r][c];
        const int64_t o = (int64_t)(i0 + r) * ldy + j0 + c;
        double v = alpha * s + beta * Y1[o];
        if (gamma != 0.0) v += gamma * Y0[o];
        Out[o] = v;
    }
}

// Partial cross products P[chunk][i][j] = sum over the chunk's rows of
// X[r][i] Y[r][j] (FP64, row-major X, Y; px, py <= kMaxBlock).  Rows staged
// 16 at a time in LDS; thread t accumulates outputs t, t + 256, ...
__global__ void __launch_bounds__(kThreads) k_xty_partial(const double* __restrict__ X, int ldx, int px,
                                                          const double* __restrict__ Y, int ldy, int py,
                                                          int64_t rows, int64_t chunk, double* __restrict__ P) {
    __shared__ double sX[16][kMaxBlock + 1];
    __shared__ double sY[16][kMaxBlock + 1];
    constexpr int NQ = kMaxBlock * kMaxBlock / kThreads;   // 36
    const int64_t ra = (int64_t)blockIdx.x * chunk;
    const int64_t rb = min(rows, ra + chunk);
    const int nout = px * py;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int64_t r0 = ra; r0 < rb; r0 += 16) {
        for (int e = threadIdx.x; e < 16 * kMaxBlock; e += kThreads) {
            const int rr = e / kMaxBlock, c = e % kMaxBlock;
            const int64_t r = r0 + rr;
            sX[rr][c] = (r < rb && c < px) ? X[r * ldx + c] : 0.0;
            sY[rr][c] = (r < rb && c < py) ? Y[r * ldy + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = threadIdx.x + q * kThreads;
            if (e < nout) {
                const int i = e / py, c = e % py;
                double s = 0.0;
#pragma unroll
                for (int rr = 0; rr < 16; ++rr) s += sX[rr][i] * sY[rr][c];
                acc[q] += s;
            }
        }
        __syncthreads();
    }
    double* out = P + (int64_t)blockIdx.x * nout;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int e = threadIdx.x + q * kThreads;
        if (e < nout) out[e] = acc[q];
    }
}

// H = (S + S^T) / 2 with S = sum of the p x p partials in chunk order:
// exactly symmetric (a Rayleigh quotient matrix X^T G X).
__global__ void k_sum_sym(const double* __restrict__ P, int nchunk, int p, double* __restrict__ H) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= p * p) return;
    const int i = e / p, j = e % p;
    double a = 0.0, b = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        a += P[(int64_t)c * p * p + i * p + j];
        b += P[(int64_t)c * p * p + j * p + i];
    }
    H[e] = 0.5 * (a + b);
}

// res[j] = ||W[:, j] - sigma_j^2 X[:, j]||_2 over `rows` rows (one block per
// column, fixed reduction order); theta[j] = sigma_j^2.
__global__ void __launch_bounds__(kThreads) k_ritz_res(const double* __restrict__ W, const double* __restrict__ X,
                                                       int ld, int64_t rows, const double* __restrict__ sig,
                                                       double* __restrict__ theta, double* __restrict__ res) {
    __shared__ double red[kThreads];
    const int j = blockIdx.x;
    const double th = sig[j] * sig[j];
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += kThreads) {
        const double d = W[r * ld + j] - th * X[r * ld + j];
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        res[j] = sqrt(red[0]);
        theta[j] = th;
    }
}

// Deflation of nl newly converged Ritz pairs (columns 0..nl-1 of X and of
// W = G_d X, Ritz values theta): G_d <- (I - L L^T) G_d (I - L L^T) with
// L = X[:, :nl], written as G_d - L N^T - N L^T with N = W - L diag(theta) / 2
// (L^T G_d L = diag(theta) for Ritz pairs).  Blocks cover the 16 x 16 tiles
// of the upper triangle (grid ntile16 (ntile16 + 1) / 2); an element is
// formed from its (min, max) index pair and written to both mirror places,
// so G_d stays exactly symmetric.
__global__ void __launch_bounds__(kThreads) k_deflate(double* __restrict__ G, int ldg, const double* __restrict__ X,
                                                      const double* __restrict__ W, int ld, int nl,
                                                      const double* __restrict__ theta) {
    __shared__ double sLi[16][kMaxBlock + 1], sNi[16][kMaxBlock + 1];
    __shared__ double sLj[16][kMaxBlock + 1], sNj[16][kMaxBlock + 1];
    const int nt = ldg / 16;
    int t = blockIdx.x, ib = 0;
    while (t >= nt - ib) {
        t -= nt - ib;
        ++ib;
    }
    const int jb = ib + t;
    for (int e = threadIdx.x; e < 16 * nl; e += kThreads) {
        const int r = e / nl, q = e % nl;
        const int64_t gi = (int64_t)(16 * ib + r) * ld + q, gj = (int64_t)(16 * jb + r) * ld + q;
        const double hq = 0.5 * theta[q];
        sLi[r][q] = X[gi];
        sNi[r][q] = W[gi] - hq * X[gi];
        sLj[r][q] = X[gj];
        sNj[r][q] = W[gj] - hq * X[gj];
    }
    __syncthreads();
    const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
    // canonical order: the element with the smaller global index first
    const bool swap = (ib == jb) && (ti > tj);
    const double* La = swap ? sLj[tj] : sLi[ti];
    const double* Na = swap ? sNj[tj] : sNi[ti];
    const double* Lb = swap ? sLi[ti] : sLj[tj];
    const double* Nb = swap ? sNi[ti] : sNj[tj];
    double s = 0.0;
    for (int q = 0; q < nl; ++q) {
        const double p1 = La[q] * Nb[q];
        const double p2 = Na[q] * Lb[q];
        s += p1 + p2;
    }
    const int64_t i = 16 * ib + ti, j = 16 * jb + tj;
    const double v = G[i * ldg + j] - s;
    __syncthreads();
    G[i * ldg + j] = v;
    if (ib != jb) G[j * ldg + i] = v;
}

// Y[r][c] -= sum_q L[r][q] C[q][c]  (rows x w, C nl x w row-major, nl <= 128)
__global__ void __launch_bounds__(kThreads) k_sub_lc(double* __restrict__ Y, int ldy, int w,
                                                     const double* __restrict__ L, int ldl, int nl,
                                                     const double* __restrict__ C, int64_t rows) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * w) return;
    const int64_t r = e / w;
    const int c = (int)(e % w);
    double s = 0.0;
    for (int q = 0; q < nl; ++q) s += L[r * ldl + q] * C[q * w + c];
    Y[r * ldy + c] -= s;
}

// Out[r][c] = In[r][c0 + c] for c < ncols, 0 for ncols <= c < wout (all rows)
__global__ void k_take_cols(const double* __restrict__ In, int ldi, int c0, int ncols, double* __restrict__ Out,
                            int wout, int64_t rows) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * wout) return;
    const int64_t r = e / wout;
    const int c = (int)(e % wout);
    Out[e] = c < ncols ? In[r * ldi + c0 + c] : 0.0;
}

// Start block of the Gram-form refresh (FP64, ldg x w, zero past n rows and
// past b columns): columns 0..kw-1 the current V (tiled layout, storage
// type), the rest a deterministic hash in [-1, 1).
template <typename T>
__global__ void k_gcf_start(double* __restrict__ X, int w, int64_t n, int64_t rows, int b,
                            const T* __restrict__ V, int ldv, int kw, uint64_t seed) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * w) return;
    const int64_t r = e / w;
    const int j = (int)(e % w);
    double v = 0.0;
    if (r < n && j < b) {
        if (j < kw) {
            v = (double)V[uvo(r, j, ldv)];
        } else {
            uint64_t h = seed ^ ((uint64_t)r * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)(j + 1) * 0xC2B2AE3D27D4EB4Full);
            h ^= h >> 33; h *= 0xff51afd7ed558ccdull; h ^= h >> 33; h *= 0xc4ceb9fe1a85ec53ull; h ^= h >> 33;
            v = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
        }
    }
    X[e] = v;
}

// Refill of the active block: columns [c0, c1) of X (leading dimension w)
// get fresh pseudo-random values on rows < n (the same hash as the start
// block, keyed by column index and `seed`); the filter, the projection
// against the locked vectors and CholQR2 that follow orthonormalise them.
__global__ void k_gcf_fill(double* __restrict__ X, int w, int64_t n, int c0, int c1, uint64_t seed) {
    const int nc = c1 - c0;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nc) return;
    const int64_t r = e / nc;
    const int j = c0 + (int)(e % nc);
    uint64_t h = seed ^ ((uint64_t)r * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)(j + 1) * 0xC2B2AE3D27D4EB4Full);
    h ^= h >> 33; h *= 0xff51afd7ed558ccdull; h ^= h >> 33; h *= 0xc4ceb9fe1a85ec53ull; h ^= h >> 33;
    X[r * w + j] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void k_start_flags(int* __restrict__ flags) {
    if (threadIdx.x < 4) flags[threadIdx.x] = 0;
}

}  // namespace isvd
