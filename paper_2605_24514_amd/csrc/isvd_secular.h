// SVD of the append core K = [[diag(s), 0], [p^T, rho]] ((k+1) x (k+1),
// Alg. A1; a column append assembles the same K on the transpose, Alg. A2)
// through the secular equation instead of Jacobi sweeps.
//
// K^T K = D + w w^T with D = diag(s_1^2, ..., s_k^2, 0) and w = [p; rho]: a
// symmetric rank-one modification of a diagonal matrix (Golub 1973; Bunch,
// Nielsen and Sorensen 1978).  Its eigenvalues lambda_i = sigma_i^2 are the
// roots of 1 + sum_j w_j^2 / (d_j - lambda) = 0, one in each gap of the
// (descending) d_j and one above d_1; the right singular vectors are the
// eigenvectors, v_i proportional to (D - lambda_i I)^{-1} w, and K v_i =
// sigma_i u_i gives the left ones.  Steps:
//   deflation  a weight |w_j| below 8 eps scale / ||w|| leaves (d_j, e_j) as
//              an eigenpair; two poles closer than 8 eps scale are merged by
//              a Givens rotation that moves the weight onto the first one
//              (scale = max(d_1, ||w||^2));
//   roots      one group of lanes per root: the root's bracket between its two poles
//              (above d_1: up to d_1 + ||w||^2), measured from the nearer
//              pole so that lambda - d_j keeps its relative accuracy,
//              bisection, then Newton steps inside the bracket until the
//              secular function is within its own rounding bound;
//   vectors    Gu and Eisenstat (1994): the weights are recomputed from the
//              computed roots, w^_j^2 = prod_i (lambda_i - d_j) /
//              prod_{i != j} (d_i - d_j), so the vectors (D - lambda_i)^{-1} w^
//              are orthogonal to working precision; the Givens rotations are
//              applied back, then W = K V.
// The left vectors u_i = K v_i / sigma_i lose orthogonality roughly as
// eps (sigma_1 / sigma_i)^2; the caller takes this path only when every
// triplet it keeps has sigma_i >= kSecularMinRatio sigma_1 (there the loss
// stays below 1e-9, far under FP32 rounding) and otherwise uses the Jacobi
// core.  All arithmetic in FP64; one workgroup per core, whose lanes share
// every O(N^2) step (roots, weights, vectors).
#pragma once
#include "isvd_common.h"
#include "isvd_jacobi.h"

namespace isvd {

constexpr double kSecularMinRatio = 1e-4;

// FP64 reciprocal: hardware estimate and two Newton steps (full precision)
__device__ inline double sec_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// scratch doubles the routine needs after its N x ldw matrix V
__host__ __device__ constexpr int secular_scratch_doubles(int nmax) { return 12 * nmax; }

// Lanes per root (and per weight, per vector norm): the largest power of two
// G <= 8 with G * NMAX <= NT, so one pass of aligned G-lane groups covers every
// root.  Group sums are DPP butterflies: every lane of a group ends with the
// same bits, so a group's control flow stays uniform.
__host__ __device__ constexpr int sec_lanes(int nmax, int nt) {
    return 8 * nmax <= nt ? 8 : 4 * nmax <= nt ? 4 : 2 * nmax <= nt ? 2 : 1;
}
template <int G>
__device__ inline double sec_gprod(double v) {
    if constexpr (G >= 2) v *= dpp_move<0xB1>(v);
    if constexpr (G >= 4) v *= dpp_move<0x4E>(v);
    if constexpr (G >= 8) v *= dpp_move<0x141>(v);
    return v;
}

// Fills V (column-major, ld ldw, columns = right singular vectors, unsorted)
// and W = K V (columns sigma_i u_i), and returns true, when the secular path
// applies (block-uniform result); otherwise returns false and leaves W and V
// untouched.  s: k singular values, descending; p: k projections; kkeep: the
// number of triplets the caller keeps at most; xs: scratch; s_cnt: 4 shared
// ints.  Launched with NT threads; N = k + 1 <= NMAX <= 128.
template <int NMAX, int NT>
__device__ inline bool secular_append_core(const double* s, const double* p, double rho, int k, int kkeep,
                                           double* W, double* V, int ldw, double* xs, int* s_cnt) {
    static_assert(NMAX <= 128, "deflation covers two poles per lane of one wave");
    constexpr int G = sec_lanes(NMAX, NT);
    constexpr int QM = (NMAX + G - 1) / G;   // poles per lane
    static_assert(G * NMAX <= NT, "one lane group per root");
    const int N = k + 1;
    const int tid = threadIdx.x;
    const double eps = 2.220446049250313e-16;
    double* dd = xs;            // kept poles, descending
    double* z = dd + N;         // their weights
    double* mu = z + N;         // root offsets from their origin pole
    double* zh = mu + N;        // recomputed weights
    double* rotc = zh + N;
    double* rots = rotc + N;
    double* lam = rots + N;     // eigenvalues (reduced roots, then deflated); later 1 / ||v_i||
    int* org = (int*)(lam + N); // origin pole of each root
    int* keep = org + N;        // original index of each kept pole
    int* defl = keep + N;       // deflated original indices
    int* rotL = defl + N;
    int* rotJ = rotL + N;
    // deflation, by the first wave: pole j is (s_j^2, p_j) for j < k and
    // (0, rho) for j = k.  A weight below tolw deflates; a pole within told
    // of the previous kept one is merged into it by a Givens rotation.  When
    // no two consecutive kept poles are that close (the usual case) the lanes
    // place the poles by ballot; otherwise lane 0 walks them in order.
    if (tid < 64) {
        const int l = tid;
        const bool v0 = l < N, v1 = l + 64 < N;
        const double d0 = l < k ? s[l] * s[l] : 0.0, w0 = v0 ? (l < k ? p[l] : rho) : 0.0;
        const double d1 = l + 64 < k ? s[l + 64] * s[l + 64] : 0.0, w1 = v1 ? (l + 64 < k ? p[l + 64] : rho) : 0.0;
        double part = w0 * w0 + w1 * w1;
        for (int o = 1; o < 64; o <<= 1) part += __shfl_xor(part, o);
        const double wn2 = part;
        const double scale = fmax(fmax(k > 0 ? s[0] * s[0] : 0.0, wn2), 1e-300);
        const double tolw = 8.0 * eps * scale / fmax(sqrt(wn2), 1e-300);
        const double told = 8.0 * eps * scale;
        const bool big0 = v0 && !(fabs(w0) <= tolw), big1 = v1 && !(fabs(w1) <= tolw);
        const unsigned long long M0 = __ballot(big0), M1 = __ballot(big1);
        const unsigned long long below = l == 0 ? 0ull : ((1ull << l) - 1ull);
        auto dpole = [&](int j) { return j < k ? s[j] * s[j] : 0.0; };
        auto highest = [](unsigned long long m) { return 63 - __clzll(m); };
        bool close = false;
        if (big0 && (M0 & below)) close = dpole(highest(M0 & below)) - d0 <= told;
        if (big1) {
            const int prev = (M1 & below) ? 64 + highest(M1 & below) : (M0 ? highest(M0) : -1);
            if (prev >= 0) close = close || dpole(prev) - d1 <= told;
        }
        if (__ballot(close) == 0ull) {
            const unsigned long long S0 = __ballot(v0 && !big0), S1 = __ballot(v1 && !big1);
            if (big0) {
                const int q = __popcll(M0 & below);
                keep[q] = l;
                dd[q] = d0;
                z[q] = w0;
            } else if (v0) {
                defl[__popcll(S0 & below)] = l;
            }
            if (big1) {
                const int q = __popcll(M0) + __popcll(M1 & below);
                keep[q] = l + 64;
                dd[q] = d1;
                z[q] = w1;
            } else if (v1) {
                defl[__popcll(S0) + __popcll(S1 & below)] = l + 64;
            }
            if (l == 0) {
                s_cnt[0] = __popcll(M0) + __popcll(M1);
                s_cnt[1] = __popcll(S0) + __popcll(S1);
                s_cnt[2] = 0;
            }
        } else if (l == 0) {
            int nd = 0, nf = 0, nr = 0;
            for (int j = 0; j < N; ++j) {
                const double dj = dpole(j);
                const double wj = j < k ? p[j] : rho;
                if (fabs(wj) <= tolw) {
                    defl[nf++] = j;
                    continue;
                }
                if (nd > 0 && dd[nd - 1] - dj <= told) {
                    const double wl = z[nd - 1];
                    const double r = sqrt(wl * wl + wj * wj);
                    rotL[nr] = keep[nd - 1];
                    rotJ[nr] = j;
                    rotc[nr] = wl / r;
                    rots[nr] = wj / r;
                    ++nr;
                    z[nd - 1] = r;
                    defl[nf++] = j;
                    continue;
                }
                keep[nd] = j;
                dd[nd] = dj;
                z[nd] = wj;
                ++nd;
            }
            s_cnt[0] = nd;
            s_cnt[1] = nf;
            s_cnt[2] = nr;
        }
    }
    __syncthreads();
    const int nd = s_cnt[0], nf = s_cnt[1], nr = s_cnt[2];
    const int gid = tid / G, sub = tid % G;
    // roots: one G-lane group per root (gid = root index); each lane keeps
    // the poles j = sub + G q and their squared weights in registers (zero
    // weights past nd)
    if (gid < nd) {
        const int i = gid;
        double dj[QM], z2[QM];
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int j = sub + G * q;
            dj[q] = j < nd ? dd[j] : -1.0;
            z2[q] = j < nd ? z[j] * z[j] : 0.0;
        }
        double lo, hi;
        int o;
        if (i == 0) {
            double sz = 0.0;
#pragma unroll
            for (int q = 0; q < QM; ++q) sz += z2[q];
            o = 0;
            lo = 0.0;
            hi = dpp_group_sum<G>(sz);
        } else {
            const double a = dd[i], half = 0.5 * (dd[i - 1] - a);
            double f = 0.0;
#pragma unroll
            for (int q = 0; q < QM; ++q) f += z2[q] * sec_rcp((dj[q] - a) - half);
            if (1.0 + dpp_group_sum<G>(f) > 0.0) {
                o = i;
                lo = 0.0;
                hi = half;
            } else {
                o = i - 1;
                lo = -half;
                hi = 0.0;
            }
        }
        const double origin = dd[o];
        const double dl = dd[i] - origin;                  // lower pole
        const double du = i > 0 ? dd[i - 1] - origin : 0.0; // upper pole (none for i = 0)
        // Each step models the terms of the poles at or below the lower pole
        // (psi) and those above it (phi) by one pole each, matching value and
        // slope at m, and moves to the model's root in the bracket:
        // C eta^2 - A eta + B = 0 with DL, DU the poles' offsets from m,
        // A = (DL + DU) f - DL DU f', B = DL DU f, C = f - DL psi' - DU phi'
        // (above the largest pole: one pole, eta = DL f / (f - DL f')).
        // A model root outside the bracket, kept by the signs of f, bisects.
        double m = 0.5 * (lo + hi);
        for (int it = 0; it < 64; ++it) {
            double sf = 0.0, sa = 0.0, sp = 0.0, sq = 0.0;
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                const double r = sec_rcp((dj[q] - origin) - m);
                const double t = z2[q] * r;
                sf += t;
                sa += fabs(t);
                if (sub + G * q >= i) sp += t * r;
                else sq += t * r;
            }
            const double f = 1.0 + dpp_group_sum<G>(sf);
            const double fa = 1.0 + dpp_group_sum<G>(sa);
            const double dpsi = dpp_group_sum<G>(sp);
            const double dphi = dpp_group_sum<G>(sq);
            if (fabs(f) <= 8.0 * eps * fa) break;
            if (f > 0.0) hi = m;
            else lo = m;
            const double DL = dl - m;
            double mn = 0.5 * (lo + hi);
            if (i == 0) {
                const double den = f - DL * dpsi;
                if (den > 0.0) {
                    const double c = m + DL * f / den;
                    if (c > lo && c < hi) mn = c;
                }
            } else {
                const double DU = du - m;
                const double A = (DL + DU) * f - DL * DU * (dpsi + dphi);
                const double B = DL * DU * f;
                const double C = f - DL * dpsi - DU * dphi;
                const double qq = 0.5 * (A + copysign(sqrt(fmax(A * A - 4.0 * B * C, 0.0)), A));
                const double c1 = C != 0.0 ? m + qq / C : lo;
                const double c2 = qq != 0.0 ? m + B / qq : lo;
                if (c1 > lo && c1 < hi) mn = c1;
                else if (c2 > lo && c2 < hi) mn = c2;
            }
            if (mn == m) break;
            m = mn;
        }
        if (sub == 0) {
            org[i] = o;
            mu[i] = m;
            lam[i] = origin + m;
        }
    }
    for (int t = tid; t < nf; t += NT) {
        const int j = defl[t];
        lam[nd + t] = j < k ? s[j] * s[j] : 0.0;
    }
    __syncthreads();
    // take this path only if every kept triplet is well above sigma_1's resolution
    if (tid < 64) {
        // reduced by the first wave
        double lmax = 0.0;
        bool finite = true;
        for (int c = tid; c < N; c += 64) {
            finite = finite && isfinite(lam[c]);
            lmax = fmax(lmax, lam[c]);
        }
        for (int o = 32; o > 0; o >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, o));
        finite = __ballot(!finite) == 0ull;
        int npos = 0, nbig = 0;
        for (int c = tid; c < N; c += 64) {
            npos += lam[c] > 0.0 ? 1 : 0;
            nbig += lam[c] >= kSecularMinRatio * kSecularMinRatio * lmax ? 1 : 0;
        }
        for (int o = 32; o > 0; o >>= 1) {
            npos += __shfl_xor(npos, o);
            nbig += __shfl_xor(nbig, o);
        }
        const int kexp = kkeep < npos ? kkeep : npos;
        if (tid == 0) s_cnt[3] = (finite && lmax > 0.0 && nbig >= kexp) ? 1 : 0;
    }
    __syncthreads();
    if (!s_cnt[3]) return false;
    // lambda_i - d_j = (d_org(i) - d_j) + mu_i
    auto diff = [&](int i, int j) { return (dd[org[i]] - dd[j]) + mu[i]; };
    // recomputed weights (one group per weight) and R[i][j] = 1 / (lambda_i - d_j) in W
    if (gid < nd) {
        const int j = gid;
        double prod = 1.0;
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int i = sub + G * q;
            if (i < nd) prod *= i == j ? diff(j, j) : diff(i, j) * sec_rcp(dd[i] - dd[j]);
        }
        prod = sec_gprod<G>(prod);
        if (sub == 0) zh[j] = copysign(sqrt(fmax(prod, 0.0)), z[j]);
    }
    for (int e = tid; e < nd * nd; e += NT) {
        const int i = e / nd, j = e - (e / nd) * nd;
        W[(size_t)i * ldw + j] = sec_rcp(diff(i, j));
    }
    for (int e = tid; e < N * ldw; e += NT) V[e] = 0.0;
    __syncthreads();
    // 1 / ||(D - lambda_i)^{-1} w^|| (one group per vector)
    if (gid < nd) {
        const int i = gid;
        double nrm = 0.0;
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int j = sub + G * q;
            if (j < nd) {
                const double v = zh[j] * W[(size_t)i * ldw + j];
                nrm += v * v;
            }
        }
        nrm = dpp_group_sum<G>(nrm);
        if (sub == 0) lam[i] = 1.0 / sqrt(nrm);
    }
    __syncthreads();
    // (D - lambda_i)^{-1} w^ = -w^_j / (lambda_i - d_j), normalised
    for (int e = tid; e < nd * nd; e += NT) {
        const int i = e / nd, j = e - (e / nd) * nd;
        V[(size_t)i * ldw + keep[j]] = -zh[j] * W[(size_t)i * ldw + j] * lam[i];
    }
    for (int t = tid; t < nf; t += NT) V[(size_t)(nd + t) * ldw + defl[t]] = 1.0;
    __syncthreads();
    // back to the original coordinates: the last rotation first
    for (int c = tid; c < N; c += NT) {
        double* vc = V + (size_t)c * ldw;
        for (int q = nr - 1; q >= 0; --q) {
            const double a = vc[rotL[q]], b = vc[rotJ[q]];
            vc[rotL[q]] = rotc[q] * a - rots[q] * b;
            vc[rotJ[q]] = rots[q] * a + rotc[q] * b;
        }
    }
    __syncthreads();
    // W = K V
    for (int e = tid; e < N * k; e += NT) {
        const int c = e / k, r = e % k;
        W[(size_t)c * ldw + r] = s[r] * V[(size_t)c * ldw + r];
    }
    // row k of W (the appended row of K times V): one G-lane group per column
    for (int c = gid; c < N; c += NT / G) {
        const double* vc = V + (size_t)c * ldw;
        double t = 0.0;
        for (int j = sub; j < k; j += G) t += p[j] * vc[j];
        t = dpp_group_sum<G>(t);
        if (sub == 0) W[(size_t)c * ldw + k] = t + rho * vc[k];
    }
    __syncthreads();
    return true;
}

}  // namespace isvd
