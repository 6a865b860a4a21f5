// Subspace-drift trackers of the angle-threshold policy (Section 3.3; the
// reference-angle metric of Section 2.4.2).
//
// theta_ref compares U_ref (stored at the last refresh, m_ref rows) with the
// current U_t restricted to those rows, re-orthonormalised.  Two k x k FP64
// matrices carry everything it needs:
//   M = U_ref^T U_t[0:m_ref, :]        H = U_t[0:m_ref, :]^T U_t[0:m_ref, :]
// and both follow every update exactly through the core's rotation of U:
//   row append / rank-1:  U_t = [U_{t-1}; new rows] Q   -> M' = M Q,  H' = Q^T H Q
//     (the appended row lies past m_ref, so only Q's first k rows act)
//   column append:        U_t = [U_{t-1}, z^] Q        -> M' = [M, a] Q,
//                                                       H' = Q^T [[H, b], [b^T, zeta]] Q
//     with a = U_ref^T z^_r, b = U_{t-1,r}^T z^_r, zeta = ||z^_r||^2 over the
//     reference rows, z^_r = (y_r - U_{t-1,r} p) / rho formed row by row.
// theta on the leading j columns (j = the scope): with H_j = R^T R
// (Cholesky), the columns of U_t[0:m_ref, :j] R^-1 are an orthonormal basis
// of the restricted span, so the principal cosines are the singular values
// of C = M_j R^-1 and theta = arccos(sigma_min(C)), evaluated as
// atan2(sqrt((1 - s)(1 + s)), s) so that small angles keep their digits.
#pragma once
#include "isvd_common.h"
#include "isvd_jacobi.h"

namespace isvd {

// One angle-policy stream's tracker work for one update.
struct Track {
    DevHeader* hdr;
    ReqScratch* rs;
    int32_t kind;
    int32_t scope;        // columns theta is measured on (0 = leading gap-separated)
    int32_t tiles;        // column append: blocks of the reference-row pass
    int32_t kc;           // row stride of M and H
    const void* Uref;
    const void* U[2];
    const void* QU;       // the core's rotation of U (rows 0..k_in, ld_out columns)
    const double* p;      // projection coefficients of a column append
    const double* S;
    const void* payload;  // y of a column append
    double* M;
    double* H;
    double* part;         // column append: per-block sums, stride 2 kc + 1
    double* scr;          // (kc + 1) x kc scratch: the product T of k_track, R of theta
};

constexpr int kTrackRows = 1024;   // reference rows per block of the column pass
// threads of the column pass: lanes [0, 128) a, [128, 256) b, lane 256 zeta
constexpr int kTrackColThreads = 320;

// Column append: per block of reference rows, a = U_ref^T z^, b = U^T z^ and
// zeta = z^^T z^ (FP64).  Rows are taken 64 at a time: four lanes form each
// row's z^, then lane c < k_ref sums U_ref[:, c] z^, lane 128 + c < k_in sums
// U[:, c] z^ and lane 256 sums z^^2 (coalesced row reads across lanes).
template <typename T>
__global__ void __launch_bounds__(kTrackColThreads) k_track_col(const Track* __restrict__ trs, const int* __restrict__ prefix,
                                                        int ntr) {
    __shared__ double sz[64];
    __shared__ double sp[kMaxCore];
    int lo = 0, hi = ntr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const Track& tr = trs[lo];
    const ReqScratch* rs = tr.rs;
    const DevHeader* hdr = tr.hdr;
    const int tile = blockIdx.x - prefix[lo];
    double* out = tr.part + (size_t)tile * (2 * tr.kc + 1);
    const int kin = rs->k_in, ldi = rs->ld_in;
    const int kref = hdr->ref_k, ldr = hdr->ref_ld;
    const int64_t mref = hdr->ref_m;
    const double inv_rho = rs->inv_rho;
    const T* U = (const T*)tr.U[rs->in_idx];
    const T* Ur = (const T*)tr.Uref;
    const T* y = (const T*)tr.payload;
    for (int c = threadIdx.x; c < kin; c += blockDim.x) sp[c] = tr.p[c];
    __syncthreads();
    const int t = threadIdx.x;
    double acc = 0.0;
    const int64_t r0 = (int64_t)tile * kTrackRows;
    const int64_t r1 = min(mref, r0 + kTrackRows);
    if (!rs->skip && inv_rho != 0.0) {
        for (int64_t rb = r0; rb < r1; rb += 64) {
            if (t < 256) {
                const int rr = t >> 2, q = t & 3;
                const int64_t r = rb + rr;
                double d = 0.0;
                if (r < r1) {
#pragma unroll 8
                    for (int c = q; c < kin; c += 4) d += (double)U[uvo(r, c, ldi)] * sp[c];
                }
                d += __shfl_xor(d, 1);
                d += __shfl_xor(d, 2);
                if (q == 0) sz[rr] = r < r1 ? ((double)y[r] - d) * inv_rho : 0.0;
            }
            __syncthreads();
            const int nr = (int)min((int64_t)64, r1 - rb);
            // the loads of a row block issue together (unrolled); the sums run in row order
            if (t < kref) {
#pragma unroll 16
                for (int rr = 0; rr < nr; ++rr) acc += (double)Ur[uvo(rb + rr, t, ldr)] * sz[rr];
            } else if (t >= 128 && t < 256 && t - 128 < kin) {
#pragma unroll 16
                for (int rr = 0; rr < nr; ++rr) acc += (double)U[uvo(rb + rr, t - 128, ldi)] * sz[rr];
            } else if (t == 256) {
                for (int rr = 0; rr < nr; ++rr) acc += sz[rr] * sz[rr];
            }
            __syncthreads();
        }
    }
    if (t < tr.kc) out[t] = t < kref ? acc : 0.0;
    if (t >= 128 && t < 256 && t - 128 < tr.kc) out[tr.kc + (t - 128)] = t - 128 < kin ? acc : 0.0;
    if (t == 256) out[2 * tr.kc] = acc;
}

// Leading gap-separated scope of a descending spectrum (Section 3.3 reading):
// the j < k maximising (s_j - s_{j+1}) / s_j if that gap is >= 5%, else k.
__device__ inline int gap_scope(const double* S, int k) {
    int best = k;
    double best_gap = -1.0;
    for (int j = 1; j < k; ++j) {
        const double g = S[j - 1] > 0.0 ? (S[j - 1] - S[j]) / S[j - 1] : 0.0;
        if (g > best_gap) { best_gap = g; best = j; }
    }
    return best_gap >= 0.05 ? best : k;
}

// LDS doubles of block_theta for scope up to kMaxBlock (about 137 KB)
__host__ __device__ constexpr size_t theta_lds_doubles() {
    return (size_t)(kMaxBlock + 1) * WideShape::LDW + 2 * kMaxBlock;
}

// theta_ref on the leading j columns from M (k_ref x k, row stride ldm) and
// H (k x k, row stride ldh) in global memory; R (j x j) is formed in the
// global scratch `Rg`.  Whole block; returns the angle on every thread.
__device__ inline double block_theta(const double* M, int ldm, const double* H, int ldh, int j, double* lds,
                                     double* Rg) {
    const int ldw = WideShape::LDW;
    double* W = lds;                                   // C column-major, (j + 1) columns
    double* R = Rg;                                    // j x j, row-major
    double* red = W + (size_t)(kMaxBlock + 1) * ldw;
    int* s_drop = (int*)(red + kMaxBlock);
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < j * j; e += nt) R[e] = H[(e / j) * ldh + (e % j)];
    __syncthreads();
    // Cholesky H_j = R^T R; a column outside the span of those before it (no
    // weight on the reference rows) is dropped and its cosine counts as zero
    const double tol = 4.0 * j * 2.220446049250313e-16;
    for (int q = 0; q < j; ++q) {
        if (tid == 0) {
            const double hqq = H[q * ldh + q];
            double d = R[q * j + q];
            for (int i = 0; i < q; ++i) d -= R[i * j + q] * R[i * j + q];
            const int drop = (d > tol * hqq && hqq > 1e-300) ? 0 : 1;
            s_drop[q] = drop;
            R[q * j + q] = drop ? 0.0 : sqrt(d);
        }
        __syncthreads();
        for (int c = q + 1 + tid; c < j; c += nt) {
            if (s_drop[q]) {
                R[q * j + c] = 0.0;
            } else {
                double s = R[q * j + c];
                for (int i = 0; i < q; ++i) s -= R[i * j + q] * R[i * j + c];
                R[q * j + c] = s / R[q * j + q];
            }
        }
        __syncthreads();
    }
    // C = M_j R^-1 row by row (forward substitution), into W column-major
    for (int e = tid; e < (j + 1) * ldw; e += nt) W[e] = 0.0;
    __syncthreads();
    for (int r = tid; r < j; r += nt) {
        for (int c = 0; c < j; ++c) {
            if (s_drop[c]) continue;
            double s = M[r * ldm + c];
            for (int l = 0; l < c; ++l) s -= W[(size_t)l * ldw + r] * R[l * j + c];
            W[(size_t)c * ldw + r] = s / R[c * j + c];
        }
    }
    __syncthreads();
    jacobi_block_fit<kMaxBlock + 1, WideShape::TPP>(W, j, ldw, 60);
    for (int c = tid; c < j; c += nt) {
        double s = 0.0;
        for (int e = 0; e < j; ++e) s += W[(size_t)c * ldw + e] * W[(size_t)c * ldw + e];
        red[c] = s_drop[c] ? 0.0 : sqrt(s);
    }
    __syncthreads();
    double smin = 1.0;
    for (int c = 0; c < j; ++c) smin = fmin(smin, red[c]);
    smin = fmax(0.0, fmin(1.0, smin));
    __syncthreads();
    return atan2(sqrt((1.0 - smin) * (1.0 + smin)), smin);
}

// One block per angle-policy stream after its update: M' and H' through the
// core's rotation of U.  The rotation Q (nq x kout) sits in LDS; M' = [M, a] Q
// is formed in chunks of kTrackChunk rows (row i of M' needs only row i of
// M, so each chunk is written back in place once computed); T = [[H, b],
// [b^T, zeta]] Q goes to the stream's global scratch, then H' = Q^T T.
// Dynamic LDS: track_lds_doubles().
constexpr int kTrackChunk = 24;
__host__ __device__ constexpr size_t track_lds_doubles() {
    return (size_t)kMaxCore * kMaxBlock + (size_t)kTrackChunk * kMaxBlock;
}
template <typename T>
__global__ void __launch_bounds__(kThreads) k_track(const Track* __restrict__ trs) {
    extern __shared__ double lds[];
    __shared__ double s_vec[2 * kMaxCore + 1];     // a [0, kMaxCore), b [kMaxCore, 2 kMaxCore), zeta
    const Track& tr = trs[blockIdx.x];
    const ReqScratch* rs = tr.rs;
    DevHeader* hdr = tr.hdr;
    if (rs->skip) return;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int kin = rs->k_in, kout = rs->k_out, ldo = rs->ld_out;
    const int kref = hdr->ref_k, kc = tr.kc;
    const bool col = tr.kind == kCol;
    const int nq = kin + (col ? 1 : 0);
    double* sQ = lds;                           // nq x kout
    double* sT = lds + kMaxCore * kMaxBlock;    // kTrackChunk x kout
    const T* Q = (const T*)tr.QU;
    for (int e = tid; e < nq * kout; e += nt) {
        const int l = e / kout, c = e % kout;
        sQ[e] = (double)Q[l * ldo + c];
    }
    // a (k_ref), b (k_in), zeta of a column append: sums of the block partials
    if (col) {
        for (int c = tid; c < 2 * kc + 1; c += nt) {
            const int dst = c < kc ? c : (c < 2 * kc ? kMaxCore + (c - kc) : 2 * kMaxCore);
            const bool keep = c < kc ? c < kMaxCore : (c < 2 * kc ? c - kc < kMaxCore : true);
            if (!keep) continue;
            double s = 0.0;
            for (int b = 0; b < tr.tiles; ++b) s += tr.part[(size_t)b * (2 * kc + 1) + c];
            s_vec[dst] = s;
        }
    }
    __syncthreads();
    // M' = [M, a] Q, kTrackChunk rows at a time
    for (int r0 = 0; r0 < kref; r0 += kTrackChunk) {
        const int nr = min(kTrackChunk, kref - r0);
        for (int e = tid; e < nr * kout; e += nt) {
            const int i = r0 + e / kout, c = e % kout;
            double s = 0.0;
            // unrolled so that the loads of M issue together; the sum runs over l in order
#pragma unroll 8
            for (int l = 0; l < kin; ++l) s += tr.M[i * kc + l] * sQ[l * kout + c];
            if (col) s += s_vec[i] * sQ[kin * kout + c];
            sT[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < nr * kout; e += nt) tr.M[(r0 + e / kout) * kc + (e % kout)] = sT[e];
        __syncthreads();
    }
    // T = [[H, b], [b^T, zeta]] Q into the scratch (row stride kc), then H' = Q^T T
    double* Tg = tr.scr;
    for (int e = tid; e < nq * kout; e += nt) {
        const int i = e / kout, c = e % kout;
        double s = 0.0;
        if (i < kin) {
#pragma unroll 8
            for (int l = 0; l < kin; ++l) s += tr.H[i * kc + l] * sQ[l * kout + c];
            if (col) s += s_vec[kMaxCore + i] * sQ[kin * kout + c];
        } else {
            for (int l = 0; l < kin; ++l) s += s_vec[kMaxCore + l] * sQ[l * kout + c];
            s += s_vec[2 * kMaxCore] * sQ[kin * kout + c];
        }
        Tg[i * kc + c] = s;
    }
    __syncthreads();
    for (int e = tid; e < kout * kout; e += nt) {
        const int i = e / kout, c = e % kout;
        double s = 0.0;
#pragma unroll 8
        for (int l = 0; l < nq; ++l) s += sQ[l * kout + i] * Tg[l * kc + c];
        tr.H[i * kc + c] = s;
    }
}

// theta_ref of each tracked stream from its updated M and H (a launch of its
// own, so that the tracker writes of k_track are visible).  Dynamic LDS:
// theta_lds_doubles().
__global__ void __launch_bounds__(WideShape::NT) k_theta_tracks(const Track* __restrict__ trs) {
    extern __shared__ double lds[];
    const Track& tr = trs[blockIdx.x];
    DevHeader* hdr = tr.hdr;
    if (tr.rs->skip) return;
    const int k = hdr->k, kref = hdr->ref_k;
    int j = tr.scope > 0 ? tr.scope : gap_scope(tr.S, k);
    j = min(j, min(k, kref));
    const double th = block_theta(tr.M, tr.kc, tr.H, tr.kc, j, lds, tr.scr);
    if (threadIdx.x == 0) hdr->angle_ref = th;
}

// Reference reset (refresh that stores U_ref, stream start): M = H = I.
__device__ inline void track_reset_body(DevHeader* hdr, double* M, double* H, int kc) {
    const int k = hdr->k;
    for (int e = threadIdx.x; e < kc * kc; e += blockDim.x) {
        const int r = e / kc, c = e % kc;
        const double v = (r == c && r < k) ? 1.0 : 0.0;
        if (M) M[e] = v;
        if (H) H[e] = v;
    }
    if (threadIdx.x == 0) {
        hdr->ref_k = k;
        hdr->ref_ld = hdr->ld;
        hdr->ref_m = hdr->m;
        hdr->angle_ref = 0.0;
    }
}
__global__ void k_track_reset(DevHeader* hdr, double* M, double* H, int kc) { track_reset_body(hdr, M, H, kc); }

// theta_ref from directly formed M (k_ref x k) and H (k x k), row stride k.
__global__ void __launch_bounds__(WideShape::NT) k_theta_direct(const double* M, const double* H, int k, int kref,
                                                           const double* S, int scope, double* out, double* Rg) {
    extern __shared__ double lds[];
    int j = scope > 0 ? scope : gap_scope(S, k);
    j = min(j, min(k, kref));
    // M has row stride k (k_ref rows), H row stride k; Rg: j x j scratch
    const double th = block_theta(M, k, H, k, j, lds, Rg);
    if (threadIdx.x == 0) *out = th;
}

// Gp[chunk] = X[rows of chunk]^T Y[rows of chunk]  (kx x ky, FP64, row stride ky);
// Y in the tiled basis layout, X too or (XROW) row-major with row stride ldx
template <typename T, bool XROW = false>
__global__ void __launch_bounds__(kThreads) k_cross_partial(const T* __restrict__ X, int ldx, int kx,
                                                            const T* __restrict__ Y, int ldy, int ky, int64_t rows,
                                                            int64_t chunk_rows, double* __restrict__ Gp) {
    __shared__ double sX[16][kMaxBlock + 1];
    __shared__ double sY[16][kMaxBlock + 1];
    const int64_t ra = (int64_t)blockIdx.x * chunk_rows;
    const int64_t rb = min(rows, ra + chunk_rows);
    const int nout = kx * ky;
    double acc[kMaxBlock * kMaxBlock / kThreads];
#pragma unroll
    for (int q = 0; q < kMaxBlock * kMaxBlock / kThreads; ++q) acc[q] = 0.0;
    for (int64_t r0 = ra; r0 < rb; r0 += 16) {
        for (int e = threadIdx.x; e < 16 * kMaxBlock; e += kThreads) {
            const int rr = e / kMaxBlock, c = e % kMaxBlock;
            const int64_t r = r0 + rr;
            sX[rr][c] = (r < rb && c < kx) ? (double)X[XROW ? r * ldx + c : uvo(r, c, ldx)] : 0.0;
            sY[rr][c] = (r < rb && c < ky) ? (double)Y[uvo(r, c, ldy)] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kMaxBlock * kMaxBlock / kThreads; ++q) {
            const int e = threadIdx.x + q * kThreads;
            if (e < nout) {
                const int i = e / ky, c = e % ky;
                double s = 0.0;
                for (int rr = 0; rr < 16; ++rr) s += sX[rr][i] * sY[rr][c];
                acc[q] += s;
            }
        }
        __syncthreads();
    }
    double* out = Gp + (int64_t)blockIdx.x * nout;
#pragma unroll
    for (int q = 0; q < kMaxBlock * kMaxBlock / kThreads; ++q) {
        const int e = threadIdx.x + q * kThreads;
        if (e < nout) out[e] = acc[q];
    }
}

// C = Q[:, 0:kq]^T P  (kq x ky, row stride ky): Q b x kq in the storage type
// (row stride ldq), P b x ky FP64 (row stride ky); one block
template <typename T>
__global__ void __launch_bounds__(kThreads) k_tn_small(const T* __restrict__ Q, int ldq, int b, int kq,
                                                       const double* __restrict__ P, int ky, double* __restrict__ C) {
    for (int e = threadIdx.x; e < kq * ky; e += kThreads) {
        const int i = e / ky, c = e % ky;
        double s = 0.0;
        for (int r = 0; r < b; ++r) s += (double)Q[r * ldq + i] * P[r * ky + c];
        C[e] = s;
    }
}

}  // namespace isvd
