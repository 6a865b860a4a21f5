// Block-wide FP64 one-sided (Hestenes) Jacobi SVD of a small square matrix
// held in LDS: the "SVD(K)" step of Algorithms A1-A3 and the Rayleigh-Ritz
// step of the refresh.
//
// W (N x N, column-major, column c at W + c*ldw) is rotated from the right
// until its columns are mutually orthogonal; the rotations are accumulated
// into J (= I on entry), so K = (W diag(1/sigma)) diag(sigma) J^T.
//
// Parallel (round-robin tournament) ordering: N' = N rounded up to even,
// N'-1 rounds of N'/2 disjoint pairs cover every pair once per sweep; a pair
// group of TPP lanes (power of two, inside one wave) reduces the dot
// products with cross-lane shuffles.  A pair is rotated iff
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
    if (j == 0) return 0;
    int x = j - 1 + r;
    if (x >= Np - 1) x -= Np - 1;
    return 1 + x;
}

// Column stride (doubles) of an order-N matrix in LDS: = 4 (mod 32), so that
// the 8-bank windows of the pair groups reading different columns spread
// over the LDS banks (the widest cores keep stride N to fit in LDS).
__host__ __device__ inline int lds_stride(int N) { return N <= 92 ? (N + 27) / 32 * 32 + 4 : N; }

// Block shape of a core of order up to NMAX: pairs of TPP lanes, the block
// just large enough for all pairs of one round.  Few lanes per pair keep the
// per-round work that every lane repeats (the rotation angle, the lane
// reductions) off most of the SIMD slots; more lanes per pair shorten each
// lane's serial dot products and rotations (a round's latency).
template <int NMAX, int TPP_ = 4>
struct JacobiShape {
    static constexpr int NPAIRS = (NMAX + 1) / 2;
    static constexpr int TPP = TPP_;
    static constexpr int EPT = (NMAX + TPP - 1) / TPP;              // elements per lane
    static constexpr int NT = ((NPAIRS * TPP + 63) / 64) * 64;      // threads per block
    // column stride of every core in the bucket: covers EPT * TPP elements,
    // so lanes load and store their elements without bounds tests (the
    // padding rows are zero and rotations keep them zero)
    static constexpr int LDW = (NMAX <= 92 ? (NMAX + 27) / 32 * 32 + 4 : NMAX) > EPT * TPP
                                   ? (NMAX <= 92 ? (NMAX + 27) / 32 * 32 + 4 : NMAX)
                                   : EPT * TPP;
};

// Shape of the block-wide Jacobi on matrices of order up to kMaxBlock + 1
// (the refresh's Rayleigh-Ritz, the orthogonality norm, the reference angle):
// eight lanes per pair keep each lane's share of a column pair in registers.
typedef JacobiShape<kMaxBlock + 1, 8> WideShape;

// Sum over aligned groups of TPP (2, 4, 8 or 16) lanes with DPP row moves:
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror.
template <int CTRL>
__device__ inline double dpp_move(double x) {
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ inline int dpp_move_int(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}

// Largest v over an aligned group of G lanes, ties to the lowest i; every
// lane of the group ends with the same pair.
template <int G>
__device__ inline void dpp_group_argmax(double& v, int& i) {
    auto take = [&](double ov, int oi) {
        if (ov > v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
        }
    };
    if constexpr (G >= 2) take(dpp_move<0xB1>(v), dpp_move_int<0xB1>(i));
    if constexpr (G >= 4) take(dpp_move<0x4E>(v), dpp_move_int<0x4E>(i));
    if constexpr (G >= 8) take(dpp_move<0x141>(v), dpp_move_int<0x141>(i));
    if constexpr (G >= 16) take(dpp_move<0x140>(v), dpp_move_int<0x140>(i));
}

template <int TPP>
__device__ inline double dpp_group_sum(double v) {
    if constexpr (TPP >= 2) v += dpp_move<0xB1>(v);
    if constexpr (TPP >= 4) v += dpp_move<0x4E>(v);
    if constexpr (TPP >= 8) v += dpp_move<0x141>(v);
    if constexpr (TPP >= 16) v += dpp_move<0x140>(v);
    return v;
}

// Returns the number of sweeps, or -1 if max_sweeps passed without convergence.
// The rotation threshold is max(N eps, tol_min): a caller whose results are
// rounded to a coarser type can stop at that type's accuracy.
// The three dot products of a pair are computed afresh (closed-form norm
// updates drift for columns much smaller than the others, and the drift can
// keep rounding-level rotations alive indefinitely).  Each lane holds its
// EPT elements of the pair's columns in registers for the round: all LDS
// loads issue before the arithmetic.  W and J have column stride
// ldw = JacobiShape<NMAX, TPP>::LDW with zero rows from N up to the stride.
// WITH_J: accumulate the rotations into J (= I on entry); without it only W
// is rotated.
// GUARD: the column stride is below the shape's EPT x TPP, so lanes touch
// rows below N only.
template <int NMAX, bool WITH_J, int TPP = 4, bool GUARD = false>
__device__ inline int jacobi_block(double* W, double* J, int N, int ldw, int max_sweeps, double tol_min = 0.0) {
    typedef JacobiShape<NMAX, TPP> S;
    const int tid = threadIdx.x;
    const int Np = N + (N & 1);
    const int npairs = Np >> 1;
    const int g = tid / S::TPP;
    const int lane = tid % S::TPP;
    const double tol = fmax((double)N * 2.220446049250313e-16, tol_min);
    const double tol2 = tol * tol;
    __shared__ int s_rot[2];
    int sweeps = -1;
    if (tid == 0) { s_rot[0] = 0; s_rot[1] = 0; }
    __syncthreads();
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        const int flag = sweep & 1;
        for (int r = 0; r < Np - 1; ++r) {
            // every lane of a pair group takes the same path (the DPP moves need them all)
            const bool live = g < npairs;
            const int a = live ? rr_slot(g, r, Np) : 0;
            const int b = live ? rr_slot(Np - 1 - g, r, Np) : 0;
            const int p = a < b ? a : b;
            const int q = a < b ? b : a;
            const bool act = live && q < N;
            double* wp = W + (size_t)p * ldw;
            double* wq = W + (size_t)q * ldw;
            double* jp = J + (size_t)p * ldw;
            double* jq = J + (size_t)q * ldw;
            double x[S::EPT], y[S::EPT], u[S::EPT], v[S::EPT];
            if (live) {   // groups without a pair this round issue no LDS traffic
#pragma unroll
            for (int i = 0; i < S::EPT; ++i) {
                const int e = lane + i * S::TPP;
                const bool in = !GUARD || e < N;
                x[i] = in ? wp[e] : 0.0;
                y[i] = in ? wq[e] : 0.0;
                if constexpr (WITH_J) {
                    u[i] = in ? jp[e] : 0.0;
                    v[i] = in ? jq[e] : 0.0;
                }
            }
            double alpha = 0.0, beta = 0.0, gam = 0.0;
#pragma unroll
            for (int i = 0; i < S::EPT; ++i) {
                alpha += x[i] * x[i];
                beta += y[i] * y[i];
                gam += x[i] * y[i];
            }
            alpha = dpp_group_sum<S::TPP>(alpha);
            beta = dpp_group_sum<S::TPP>(beta);
            gam = dpp_group_sum<S::TPP>(gam);
            if (act && gam * gam > tol2 * alpha * beta) {
                // t = tan of the rotation angle, the smaller root of
                // t^2 + 2 zeta t - 1 = 0 with zeta = (beta - alpha) / (2 gamma),
                // written without forming zeta
                const double d = beta - alpha;
                const double t = (d >= 0.0 ? 2.0 * gam : -2.0 * gam) / (fabs(d) + sqrt(d * d + 4.0 * gam * gam));
                const double c = rsqrt(1.0 + t * t);
                const double sn = c * t;
#pragma unroll
                for (int i = 0; i < S::EPT; ++i) {
                    const int e = lane + i * S::TPP;
                    if (GUARD && e >= N) continue;
                    wp[e] = c * x[i] - sn * y[i];
                    wq[e] = sn * x[i] + c * y[i];
                    if constexpr (WITH_J) {
                        jp[e] = c * u[i] - sn * v[i];
                        jq[e] = sn * u[i] + c * v[i];
                    }
                }
                if (lane == 0) s_rot[flag] = 1;
            }
            }
            __syncthreads();
        }
        const int rotated = s_rot[flag];
        __syncthreads();
        if (tid == 0) s_rot[flag] = 0;
        if (rotated == 0) { sweeps = sweep; break; }
    }
    __syncthreads();
    return sweeps;
}

// jacobi_block without J on an order-N matrix laid out for the shape of
// order NMAX_ALL (stride ldw, zero rows from N on): each lane holds only the
// elements of rows below the smallest of 32, 64, 96 and NMAX_ALL that covers
// N.  The rows dropped are zero in both columns of every pair, so the dot
// products lose only terms +-0 and every result is bitwise that of the
// NMAX_ALL shape, with a fraction of its LDS reads and writes.
template <int NMAX_ALL, int TPP>
__device__ inline int jacobi_block_fit(double* W, int N, int ldw, int max_sweeps, double tol_min = 0.0) {
    static_assert(NMAX_ALL > 96, "shape of the widest order");
    if (N <= 32) return jacobi_block<32, false, TPP>(W, nullptr, N, ldw, max_sweeps, tol_min);
    if (N <= 64) return jacobi_block<64, false, TPP>(W, nullptr, N, ldw, max_sweeps, tol_min);
    if (N <= 96) return jacobi_block<96, false, TPP>(W, nullptr, N, ldw, max_sweeps, tol_min);
    return jacobi_block<NMAX_ALL, false, TPP>(W, nullptr, N, ldw, max_sweeps, tol_min);
}

// Singular values of W's columns sorted non-increasing (ties: lower column
// first): sig_sorted[j] and perm[j] = column holding the j-th value.
__device__ inline void jacobi_sort(const double* W, int N, int ldw, double* sig_sorted, int* perm, double* tmp) {
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    for (int c = tid; c < N; c += nt) {
        const double* w = W + (size_t)c * ldw;
        double s = 0.0;
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
}

// After jacobi_block with J: sigma sorted, perm, and sgn[j] = +-1 making the
// largest-magnitude entry of the j-th right vector (column perm[j] of J)
// positive (first one on ties).
__device__ inline void jacobi_finish(const double* W, const double* J, int N, int ldw, double* sig_sorted,
                                     int* perm, double* sgn, double* tmp) {
    jacobi_sort(W, N, ldw, sig_sorted, perm, tmp);
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    for (int jj = tid; jj < N; jj += nt) {
        const double* v = J + (size_t)perm[jj] * ldw;
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
