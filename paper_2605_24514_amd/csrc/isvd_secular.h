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
//   roots      one thread per root: the root's bracket between its two poles
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
// core.  All arithmetic in FP64; one workgroup per core.
#pragma once
#include "isvd_common.h"

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

// Fills V (column-major, ld ldw, columns = right singular vectors, unsorted)
// and W = K V (columns sigma_i u_i), and returns true, when the secular path
// applies (block-uniform result); otherwise returns false and leaves W and V
// untouched.  s: k singular values, descending; p: k projections; kkeep: the
// number of triplets the caller keeps at most; xs: scratch; s_cnt: 4 shared ints.
__device__ inline bool secular_append_core(const double* s, const double* p, double rho, int k, int kkeep,
                                           double* W, double* V, int ldw, double* xs, int* s_cnt) {
    const int N = k + 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    const double eps = 2.220446049250313e-16;
    double* dd = xs;            // kept poles, descending
    double* z = dd + N;         // their weights
    double* mu = z + N;         // root offsets from their origin pole
    double* zh = mu + N;        // recomputed weights
    double* rotc = zh + N;
    double* rots = rotc + N;
    double* lam = rots + N;     // eigenvalues, reduced roots then deflated
    int* org = (int*)(lam + N); // origin pole of each root
    int* keep = org + N;        // original index of each kept pole
    int* defl = keep + N;       // deflated original indices
    int* rotL = defl + N;
    int* rotJ = rotL + N;
    if (tid == 0) {
        double wn2 = rho * rho;
        for (int j = 0; j < k; ++j) wn2 += p[j] * p[j];
        const double d1 = s[0] * s[0];
        const double scale = fmax(fmax(d1, wn2), 1e-300);
        const double tolw = 8.0 * eps * scale / fmax(sqrt(wn2), 1e-300);
        const double told = 8.0 * eps * scale;
        int nd = 0, nf = 0, nr = 0;
        for (int j = 0; j < N; ++j) {
            const double dj = j < k ? s[j] * s[j] : 0.0;
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
    __syncthreads();
    const int nd = s_cnt[0], nf = s_cnt[1], nr = s_cnt[2];
    // roots
    for (int i = tid; i < nd; i += nt) {
        double lo, hi;
        int o;
        if (i == 0) {
            double sz = 0.0;
            for (int j = 0; j < nd; ++j) sz += z[j] * z[j];
            o = 0;
            lo = 0.0;
            hi = sz;
        } else {
            const double a = dd[i], half = 0.5 * (dd[i - 1] - a);
            double f = 1.0;
            for (int j = 0; j < nd; ++j) f += z[j] * z[j] * sec_rcp((dd[j] - a) - half);
            if (f > 0.0) {
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
        // f, f' and the rounding bound of f (1 + sum of |terms|)
        auto fval = [&](double m, double* fp, double* fa) {
            double f = 1.0, d = 0.0, a = 1.0;
            for (int j = 0; j < nd; ++j) {
                const double r = sec_rcp((dd[j] - origin) - m);
                const double t = z[j] * z[j] * r;
                f += t;
                a += fabs(t);
                d += t * r;
            }
            *fp = d;
            *fa = a;
            return f;
        };
        double m = 0.5 * (lo + hi), fp, fa;
        for (int it = 0; it < 20; ++it) {
            if (fval(m, &fp, &fa) > 0.0) hi = m;
            else lo = m;
            m = 0.5 * (lo + hi);
        }
        // Newton with the bracket as safeguard (a step that leaves it bisects),
        // until f is within its own rounding error
        for (int it = 0; it < 40; ++it) {
            const double f = fval(m, &fp, &fa);
            if (fabs(f) <= 8.0 * eps * fa) break;
            if (f > 0.0) hi = m;
            else lo = m;
            double mn = m - f / fp;
            if (!(mn > lo && mn < hi)) mn = 0.5 * (lo + hi);
            if (mn == m) break;
            m = mn;
        }
        org[i] = o;
        mu[i] = m;
        lam[i] = origin + m;
    }
    for (int t = tid; t < nf; t += nt) {
        const int j = defl[t];
        lam[nd + t] = j < k ? s[j] * s[j] : 0.0;
    }
    __syncthreads();
    // take this path only if every kept triplet is well above sigma_1's resolution
    if (tid == 0) {
        double lmax = 0.0;
        bool finite = true;
        for (int c = 0; c < N; ++c) {
            finite = finite && isfinite(lam[c]);
            lmax = fmax(lmax, lam[c]);
        }
        int npos = 0, nbig = 0;
        for (int c = 0; c < N; ++c) {
            npos += lam[c] > 0.0 ? 1 : 0;
            nbig += lam[c] >= kSecularMinRatio * kSecularMinRatio * lmax ? 1 : 0;
        }
        const int kexp = kkeep < npos ? kkeep : npos;
        s_cnt[3] = (finite && lmax > 0.0 && nbig >= kexp) ? 1 : 0;
    }
    __syncthreads();
    if (!s_cnt[3]) return false;
    // lambda_i - d_j = (d_org(i) - d_j) + mu_i
    auto diff = [&](int i, int j) { return (dd[org[i]] - dd[j]) + mu[i]; };
    for (int j = tid; j < nd; j += nt) {
        double prod = diff(j, j);
        for (int i = 0; i < nd; ++i)
            if (i != j) prod *= diff(i, j) / (dd[i] - dd[j]);
        zh[j] = copysign(sqrt(fmax(prod, 0.0)), z[j]);
    }
    for (int e = tid; e < N * ldw; e += nt) V[e] = 0.0;
    __syncthreads();
    for (int i = tid; i < nd; i += nt) {
        double nrm = 0.0;
        for (int j = 0; j < nd; ++j) {
            const double v = zh[j] / diff(i, j);
            nrm += v * v;
        }
        const double inv = 1.0 / sqrt(nrm);
        // (D - lambda_i)^{-1} w^ = -w^_j / (lambda_i - d_j)
        for (int j = 0; j < nd; ++j) V[(size_t)i * ldw + keep[j]] = -zh[j] / diff(i, j) * inv;
    }
    for (int t = tid; t < nf; t += nt) V[(size_t)(nd + t) * ldw + defl[t]] = 1.0;
    __syncthreads();
    // back to the original coordinates: the last rotation first
    for (int c = tid; c < N; c += nt) {
        double* vc = V + (size_t)c * ldw;
        for (int q = nr - 1; q >= 0; --q) {
            const double a = vc[rotL[q]], b = vc[rotJ[q]];
            vc[rotL[q]] = rotc[q] * a - rots[q] * b;
            vc[rotJ[q]] = rots[q] * a + rotc[q] * b;
        }
    }
    __syncthreads();
    // W = K V
    for (int e = tid; e < N * k; e += nt) {
        const int c = e / k, r = e % k;
        W[(size_t)c * ldw + r] = s[r] * V[(size_t)c * ldw + r];
    }
    for (int c = tid; c < N; c += nt) {
        const double* vc = V + (size_t)c * ldw;
        double t = rho * vc[k];
        for (int j = 0; j < k; ++j) t += p[j] * vc[j];
        W[(size_t)c * ldw + k] = t;
    }
    __syncthreads();
    return true;
}

}  // namespace isvd
