/*
 * Oracle (test infrastructure only): plain FP64 one-sided Jacobi SVD.
 *
 * Computes the thin SVD A = U diag(S) V^T of a real m x n matrix with m >= n
 * (the caller transposes wide matrices).  This is the full SVD the paper's
 * background section defines (singular values non-increasing, U and V with
 * orthonormal columns); the paper calls a library SVD for the small core of
 * every update and for every refresh, and this routine stands in for both.
 *
 * Method (written from the published descriptions, not from any code):
 *  - Tall inputs (m > n) are first reduced with an unpivoted Householder QR,
 *    A = Q R, and Jacobi runs on the n x n factor R (the QR-preconditioned
 *    one-sided Jacobi of Drmac and Veselic); U = Q [U_R; 0].
 *  - One-sided (Hestenes) Jacobi on the columns g_1..g_n of the working
 *    matrix: cyclic by rows, pairs (p,q) with p < q.  A pair is rotated iff
 *    |g_p.g_q| > tol * ||g_p|| ||g_q|| with tol = n * eps; the rotation
 *    makes the two columns orthogonal.  Sweeps stop after one with no
 *    rotation, or fail after max_sweeps.
 *  - sigma_j = ||g_j||, u_j = g_j / sigma_j, v_j = accumulated rotations.
 *  - Triplets sorted by non-increasing sigma; ties keep the lower index.
 *  - Sign convention: the entry of largest magnitude of each v_j (first one
 *    on ties) is made positive, flipping u_j along with it.
 *
 * Storage: A, U, V are row-major with leading dimensions lda, ldu, ldv.
 * Returns the number of sweeps used, or -1 if max_sweeps was reached, or
 * -2 on bad arguments / allocation failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

static double dot(const double* a, const double* b, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Householder QR of the column-major m x n matrix Q (m > n) in place: on exit
 * the upper triangle holds R and the part below the diagonal of column j holds
 * the reflector v_j (implicit leading 1), with tau[j] its scale: H_j = I - tau v v^T. */
static void householder_qr(double* Q, int64_t m, int64_t n, double* tau) {
    for (int64_t j = 0; j < n; ++j) {
        double* col = Q + j * m;
        double alpha = col[j];
        double xnorm = sqrt(dot(col + j + 1, col + j + 1, m - j - 1));
        if (xnorm == 0.0) { tau[j] = 0.0; continue; }
        double beta = -copysign(hypot(alpha, xnorm), alpha);
        tau[j] = (beta - alpha) / beta;
        double scale = 1.0 / (alpha - beta);
        for (int64_t i = j + 1; i < m; ++i) col[i] *= scale;
        col[j] = beta;
        for (int64_t c = j + 1; c < n; ++c) {
            double* cc = Q + c * m;
            double w = cc[j] + dot(col + j + 1, cc + j + 1, m - j - 1);
            w *= tau[j];
            cc[j] -= w;
            for (int64_t i = j + 1; i < m; ++i) cc[i] -= w * col[i];
        }
    }
}

/* Y <- H_0 H_1 ... H_{n-1} Y for the column-major m x ncol matrix Y. */
static void apply_q(const double* Qr, const double* tau, int64_t m, int64_t n, double* Y, int64_t ncol) {
    for (int64_t j = n - 1; j >= 0; --j) {
        if (tau[j] == 0.0) continue;
        const double* v = Qr + j * m;
        for (int64_t c = 0; c < ncol; ++c) {
            double* y = Y + c * m;
            double w = y[j] + dot(v + j + 1, y + j + 1, m - j - 1);
            w *= tau[j];
            y[j] -= w;
            for (int64_t i = j + 1; i < m; ++i) y[i] -= w * v[i];
        }
    }
}

/* One-sided Jacobi on the column-major L x n matrix G, accumulating the
 * rotations into the column-major n x n matrix V (initialised to I here). */
static int hestenes(double* G, int64_t L, int64_t n, double* V, int max_sweeps) {
    const double tol = (double)n * DBL_EPSILON;
    for (int64_t i = 0; i < n * n; ++i) V[i] = 0.0;
    for (int64_t i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        int64_t rotated = 0;
        for (int64_t p = 0; p < n - 1; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                double* gp = G + p * L;
                double* gq = G + q * L;
                double alpha = dot(gp, gp, L);
                double beta = dot(gq, gq, L);
                double gamma = dot(gp, gq, L);
                if (!(fabs(gamma) > tol * sqrt(alpha) * sqrt(beta))) continue;
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t;
                if (fabs(zeta) > 1e150) t = 0.5 / zeta;
                else t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = c * t;
                for (int64_t i = 0; i < L; ++i) {
                    double a = gp[i], b = gq[i];
                    gp[i] = c * a - s * b;
                    gq[i] = s * a + c * b;
                }
                double* vp = V + p * n;
                double* vq = V + q * n;
                for (int64_t i = 0; i < n; ++i) {
                    double a = vp[i], b = vq[i];
                    vp[i] = c * a - s * b;
                    vq[i] = s * a + c * b;
                }
                ++rotated;
            }
        }
        if (rotated == 0) return sweep;
    }
    return -1;
}

int oracle_jacobi_svd(int64_t m, int64_t n, const double* A, int64_t lda,
                      double* U, int64_t ldu, double* S, double* V, int64_t ldv,
                      int max_sweeps) {
    if (m < n || n < 1 || lda < n || ldu < n || ldv < n) return -2;
    const int tall = m > n;
    const int64_t L = tall ? n : m;
    double* Qr = NULL;
    double* tau = NULL;
    double* G = (double*)calloc((size_t)(L * n), sizeof(double));
    double* Vc = (double*)malloc(sizeof(double) * (size_t)(n * n));
    double* sig = (double*)malloc(sizeof(double) * (size_t)n);
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!G || !Vc || !sig || !order) { free(G); free(Vc); free(sig); free(order); return -2; }
    if (tall) {
        Qr = (double*)malloc(sizeof(double) * (size_t)(m * n));
        tau = (double*)malloc(sizeof(double) * (size_t)n);
        if (!Qr || !tau) { free(G); free(Vc); free(sig); free(order); free(Qr); free(tau); return -2; }
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) Qr[j * m + i] = A[i * lda + j];
        householder_qr(Qr, m, n, tau);
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i <= j; ++i) G[j * n + i] = Qr[j * m + i];
    } else {
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) G[j * m + i] = A[i * lda + j];
    }
    int sweeps = hestenes(G, L, n, Vc, max_sweeps);
    for (int64_t j = 0; j < n; ++j) {
        sig[j] = sqrt(dot(G + j * L, G + j * L, L));
        order[j] = j;
    }
    /* stable insertion sort by non-increasing sigma */
    for (int64_t a = 1; a < n; ++a) {
        int64_t key = order[a];
        int64_t b = a - 1;
        while (b >= 0 && sig[order[b]] < sig[key]) { order[b + 1] = order[b]; --b; }
        order[b + 1] = key;
    }
    /* normalised left vectors of the working matrix, in sorted order */
    double* W = (double*)calloc((size_t)(m * n), sizeof(double));
    if (!W) { free(G); free(Vc); free(sig); free(order); free(Qr); free(tau); return -2; }
    for (int64_t jj = 0; jj < n; ++jj) {
        int64_t j = order[jj];
        double s = sig[j];
        for (int64_t i = 0; i < L; ++i) W[jj * m + i] = s > 0.0 ? G[j * L + i] / s : 0.0;
    }
    if (tall) apply_q(Qr, tau, m, n, W, n);
    for (int64_t jj = 0; jj < n; ++jj) {
        int64_t j = order[jj];
        const double* vj = Vc + j * n;
        int64_t imax = 0;
        for (int64_t i = 1; i < n; ++i)
            if (fabs(vj[i]) > fabs(vj[imax])) imax = i;
        double sgn = vj[imax] < 0.0 ? -1.0 : 1.0;
        S[jj] = sig[j];
        for (int64_t i = 0; i < n; ++i) V[i * ldv + jj] = sgn * vj[i];
        for (int64_t i = 0; i < m; ++i) U[i * ldu + jj] = sgn * W[jj * m + i];
    }
    free(W); free(G); free(Vc); free(sig); free(order); free(Qr); free(tau);
    return sweeps;
}
