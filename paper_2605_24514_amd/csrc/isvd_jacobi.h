// Block-wide FP64 one-sided (Hestenes) Jacobi SVD of a small square matrix
// held in LDS: the "SVD(K)" step of Algorithms A1-A3 and the Rayleigh-Ritz
// step of the refresh.
//
// W (N x N, column-major, column c at W + c*N) is rotated from the right
// until its columns are mutually orthogonal; the rotations are accumulated
// into J (= I on entry), so K = (W diag(1/sigma)) diag(sigma) J^T.
//
// Parallel (round-robin tournament) ordering: N' = N rounded up to even,
// N'-1 rounds of N'/2 disjoint pairs cover every pair once per sweep; a pair
// group of `tpp` lanes (power of two, inside one wave) reduces the dot
// product with cross-lane shuffles.  Column norms are cached and updated in
// closed form (alpha' = alpha - t gamma, beta' = beta + t gamma), refreshed
// exactly at the start of every sweep.  A pair is rotated iff
// |gamma| > N eps sqrt(alpha beta); sweeps stop after one without rotation.
#pragma once
#include "isvd_common.h"

namespace isvd {

__device__ inline double group_sum(double v, int tpp) {
    for (int o = tpp >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Slot of position j in round r of the circle method on Np players.
__device__ inline int rr_slot(int j, int r, int Np) {
    return j == 0 ? 0 : 1 + (j - 1 + r) % (Np - 1);
}

// Returns the number of sweeps, or -1 if max_sweeps passed without convergence.
__device__ inline int jacobi_block(double* W, double* J, double* nrm, int N, int max_sweeps) {
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int Np = N + (N & 1);
    const int npairs = Np >> 1;
    int tpp = 64;
    while (tpp > 1 && tpp * npairs > nt) tpp >>= 1;
    const int g = tid / tpp;
    const int lane = tid % tpp;
    const double tol = (double)N * 2.220446049250313e-16;
    __shared__ int s_rot;
    int sweeps = -1;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        for (int c = tid; c < N; c += nt) {
            double s = 0.0;
            const double* w = W + (size_t)c * N;
            for (int e = 0; e < N; ++e) s += w[e] * w[e];
            nrm[c] = s;
        }
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int r = 0; r < Np - 1; ++r) {
            if (g < npairs) {
                int a = rr_slot(g, r, Np);
                int b = rr_slot(Np - 1 - g, r, Np);
                int p = a < b ? a : b;
                int q = a < b ? b : a;
                if (q < N) {
                    double* wp = W + (size_t)p * N;
                    double* wq = W + (size_t)q * N;
                    double gam = 0.0;
                    for (int e = lane; e < N; e += tpp) gam += wp[e] * wq[e];
                    gam = group_sum(gam, tpp);
                    double alpha = nrm[p], beta = nrm[q];
                    if (fabs(gam) > tol * sqrt(alpha) * sqrt(beta)) {
                        double zeta = (beta - alpha) / (2.0 * gam);
                        double t = fabs(zeta) > 1e150 ? 0.5 / zeta
                                                      : copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        double c = 1.0 / sqrt(1.0 + t * t);
                        double s = c * t;
                        double* jp = J + (size_t)p * N;
                        double* jq = J + (size_t)q * N;
                        for (int e = lane; e < N; e += tpp) {
                            double x = wp[e], y = wq[e];
                            wp[e] = c * x - s * y;
                            wq[e] = s * x + c * y;
                            double u = jp[e], v = jq[e];
                            jp[e] = c * u - s * v;
                            jq[e] = s * u + c * v;
                        }
                        if (lane == 0) {
                            nrm[p] = alpha - t * gam;
                            nrm[q] = beta + t * gam;
                            s_rot = 1;
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (s_rot == 0) { sweeps = sweep; break; }
        __syncthreads();
    }
    __syncthreads();
    return sweeps;
}

// After jacobi_block: sigma sorted non-increasing (ties: lower column first),
// perm[j] = column of W / J holding the j-th triplet, sgn[j] = +-1 making the
// largest-magnitude entry of the j-th right vector positive.
__device__ inline void jacobi_finish(const double* W, const double* J, int N, double* sig_sorted,
                                     int* perm, double* sgn, double* tmp) {
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    for (int c = tid; c < N; c += nt) {
        double s = 0.0;
        const double* w = W + (size_t)c * N;
        for (int e = 0; e < N; ++e) s += w[e] * w[e];
        tmp[c] = sqrt(s);
    }
    __syncthreads();
    for (int c = tid; c < N; c += nt) {
        double sc = tmp[c];
        int rank = 0;
        for (int d = 0; d < N; ++d) {
            double sd = tmp[d];
            rank += (sd > sc || (sd == sc && d < c)) ? 1 : 0;
        }
        perm[rank] = c;
        sig_sorted[rank] = sc;
    }
    __syncthreads();
    for (int jj = tid; jj < N; jj += nt) {
        const double* v = J + (size_t)perm[jj] * N;
        int imax = 0;
        double vmax = fabs(v[0]);
        for (int e = 1; e < N; ++e) {
            double a = fabs(v[e]);
            if (a > vmax) { vmax = a; imax = e; }
        }
        sgn[jj] = v[imax] < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();
}

}  // namespace isvd
