// Update kernels of the engine loop (Algorithm 1): projection with one
// re-orthogonalisation pass, the FP64 core SVD, truncation, and the basis
// rotations.  Every kernel serves a list of requests of one rank bucket
// (KC = capacity of the bucket, a multiple of 4), one or more blocks each.
#pragma once
#include "isvd_common.h"
#include "isvd_jacobi.h"
#include "isvd_secular.h"

namespace isvd {

template <typename T> struct V4;
template <> struct V4<float> { typedef float4 type; };
template <> struct V4<double> { typedef double4 type; };

template <typename T>
__device__ inline void load4(const T* p, double out[4]) {
    typename V4<T>::type v = *reinterpret_cast<const typename V4<T>::type*>(p);
    out[0] = (double)v.x; out[1] = (double)v.y; out[2] = (double)v.z; out[3] = (double)v.w;
}
template <typename T> struct GV4;
template <> struct GV4<float> { typedef gvec_f4 type; };
template <> struct GV4<double> { typedef gvec_d4 type; };
template <typename T>
__device__ inline void load4(const ISVD_GLOBAL T* p, double out[4]) {
    typename GV4<T>::type v = *reinterpret_cast<const ISVD_GLOBAL typename GV4<T>::type*>(p);
    out[0] = (double)v.x; out[1] = (double)v.y; out[2] = (double)v.z; out[3] = (double)v.w;
}

// Request owning block b: the last r with prefix[r] <= b.
__device__ inline int find_req(const int* prefix, int nreq, int b) {
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline const void* basis_cur(const Req& rq, bool useU, int cur) {
    return useU ? rq.U[cur] : rq.V[cur];
}

// ---------------------------------------------------------------------------
// Projection (Section 2.2.1, eq. row-residual) with one classical
// Gram-Schmidt re-orthogonalisation pass, over row tiles of the projected
// basis X (V for a row append, U for a column append) with payload y:
//   pass 1: p1 = X^T y, ||y||^2 and the count of non-finite y entries
//   pass 2: z1 = y - X p1 per row, p2 = X^T z1, ||z1||^2
// Then p = p1 + p2 and rho^2 = ||z1||^2 - ||p2||^2 (X has orthonormal
// columns), so the residual z = y - X p never has to be stored: the rotation
// recomputes it per row.  Each block writes its FP64 partial sums (stride
// KC + 2: [0, k) the projection, [KC] the squared norm, [KC + 1] the
// non-finite count); the next launch adds the partials in block order
// (deterministic, independent of the batch), so no block waits for another.
// LDS (doubles) of one projection block of bucket KC
template <int KC>
__host__ __device__ constexpr int proj_lds_doubles() { return (kThreads / (KC / 4)) * (KC + 2) + KC; }

// Projection tile `tile` (rows [tile kProjTile, ...)) of one request.
template <typename T, int KC, int PASS>
__device__ __attribute__((always_inline)) inline void proj_tile(const Req* __restrict__ rqp, int tile, double* lds) {
    constexpr int TPR = KC / 4;                  // lanes per row (4 columns each)
    constexpr int RPB = kThreads / TPR;          // rows per block step
    constexpr int SP = KC + 2;
    constexpr int UNR = 4;                       // row steps in flight per lane
    const Req& rq = *rqp;
    double (*sacc)[SP] = reinterpret_cast<double (*)[SP]>(lds);
    double* sp1 = lds + RPB * SP;
    const ISVD_GLOBAL DevHeader* hdr = gmem(rq.hdr);
    const int k = hdr->k, ld = hdr->ld, cur = hdr->cur;
    const bool useU = rq.kind == kCol;
    const ISVD_GLOBAL T* X = gmem((const T*)basis_cur(rq, useU, cur));
    const int64_t rows = useU ? rq.m : rq.n;
    const ISVD_GLOBAL T* y = gmem((const T*)rq.payload);
    if (PASS == 2) {
        // p1: pass 1's partials in block order
        for (int c = threadIdx.x; c < KC; c += kThreads) {
            double s1 = 0.0;
            if (c < k)
                for (int t = 0; t < rq.proj_tiles; ++t) s1 += gmem(rq.partials)[(size_t)t * SP + c];
            sp1[c] = s1;
        }
        __syncthreads();
    }
    const int64_t r0 = (int64_t)tile * kProjTile;
    const int64_t r1 = min(rows, r0 + kProjTile);
    const int lane = threadIdx.x % TPR, grp = threadIdx.x / TPR;
    const int c0 = lane * 4;
    double cm[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) cm[q] = c0 + q < k ? 1.0 : 0.0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    double sq = 0.0, bad = 0.0;
    // every lane of a row group runs the same trip count (pass 2 shuffles)
    for (int64_t b0 = r0; b0 < r1; b0 += (int64_t)RPB * UNR) {
        double xv[UNR][4], yv[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t r = b0 + grp + (int64_t)u * RPB;
            const bool live = r < r1;
            if (live && c0 < k) {
                load4<T>(X + uvo(r, c0, ld), xv[u]);
#pragma unroll
                for (int q = 0; q < 4; ++q) xv[u][q] *= cm[q];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) xv[u][q] = 0.0;
            }
            yv[u] = live ? (double)y[r] : 0.0;
        }
        if (PASS == 1) {
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] += yv[u] * xv[u][q];
                if (lane == 0) {
                    sq += yv[u] * yv[u];
                    if (!isfinite(yv[u])) bad += 1.0;
                }
            }
        } else {
            double d[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u)
                d[u] = xv[u][0] * sp1[c0] + xv[u][1] * sp1[c0 + 1] + xv[u][2] * sp1[c0 + 2] + xv[u][3] * sp1[c0 + 3];
#pragma unroll
            for (int o = TPR >> 1; o > 0; o >>= 1)
#pragma unroll
                for (int u = 0; u < UNR; ++u) d[u] += __shfl_xor(d[u], o);
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const bool live = b0 + grp + (int64_t)u * RPB < r1;
                const double z1 = live ? yv[u] - d[u] : 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] += xv[u][q] * z1;
                if (lane == 0) sq += z1 * z1;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) sacc[grp][c0 + q] = acc[q];
    if (lane == 0) {
        sacc[grp][KC] = sq;
        sacc[grp][KC + 1] = bad;
    }
    __syncthreads();
    ISVD_GLOBAL double* part = gmem(PASS == 1 ? rq.partials : rq.partials2) + (size_t)tile * SP;
    for (int c = threadIdx.x; c < SP; c += kThreads) {
        double s1 = 0.0;
        for (int gg = 0; gg < RPB; ++gg) s1 += sacc[gg][c];
        part[c] = s1;
    }
}

// One block's part of a projection launch: block `bid` of the request list
// (reqs, prefix, nreq); lds: proj_lds_doubles<KC>() doubles.
template <typename T, int KC, int PASS>
__device__ __attribute__((always_inline)) inline void proj_block(const Req* __restrict__ reqs,
                                                                 const int* __restrict__ prefix, int nreq, int bid,
                                                                 double* lds) {
    // a grid sized for more tiles than this launch has (a captured tick,
    // sized for the streams' capacity) leaves the extra blocks idle
    if (bid >= prefix[nreq]) return;
    const int ri = find_req(prefix, nreq, bid);
    proj_tile<T, KC, PASS>(reqs + ri, bid - prefix[ri], lds);
}

template <typename T, int KC, int PASS>
__global__ void __launch_bounds__(kThreads) k_proj(const Req* __restrict__ reqs, const int* __restrict__ prefix,
                                                   int nreq) {
    __shared__ double lds[proj_lds_doubles<KC>()];
    proj_block<T, KC, PASS>(reqs, prefix, nreq, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Core: assemble K, its FP64 SVD, sort, sign, truncate, and the rotation
// matrices for U and V.
//   row append   K = [[Sigma, 0], [p, rho]]       (Alg. A1, (k+1) x (k+1))
//   column app.  same K on the transpose           (Alg. A2)
//   rank-1       K = Sigma + delta s_u s_v^T       (Alg. A3, k x k; s_v = row j of V)
// Rotation matrices (row-major, ld_out columns, zero beyond k_out):
//   row:    U' = [[U,0],[0,1]] U_K -> QU = U_K[0:k,:], new row m of U' = U_K[k,:]
//           V' = [V z^]      V_K -> QV = V_K[0:k+1,:] (row k multiplies z^)
//   column: U' = [U z^]      V_K -> QU = V_K[0:k+1,:]
//           V' = [[V,0],[0,1]] U_K -> QV = U_K[0:k,:], new row n of V' = U_K[k,:]
//   rank-1: QU = U_K, QV = V_K
// Truncation keeps min(k_keep, order) triplets and never a zero singular
// value after an append; the rank-1 update keeps the rank.
// One-sided Jacobi rotates the columns of W = K; U_K = W diag(1/sigma).
// FP64 storage accumulates the rotations (V_K = J).  FP32 storage does not:
// V_K = K^T U_K diag(1/sigma), evaluated from K's sparsity in O(N^2); its
// loss of orthogonality, about N eps64 sigma_1 / sigma_j, stays far below
// FP32 rounding for every kept triplet.
// FP32 storage, appends, buckets up to 64: the secular-equation SVD of the
// arrow-shaped K (isvd_secular.h) replaces the Jacobi sweeps whenever every
// kept triplet has sigma >= 1e-4 sigma_1; it leaves V_K in J and W = K V_K.
// One block per request; dynamic LDS = (matrices N ldw + small arrays) doubles
// with ldw the bucket's padded column stride, N <= kMaxCore (core_lds_doubles).
typedef double core_v4d __attribute__((ext_vector_type(4)));

template <int KC>
struct CoreShape {
    static constexpr int NMAX = (KC < kMaxCore - 1 ? KC : kMaxCore - 1) + 1;
    // eight lanes per pair for the 33-, 65- and 129-column cores (shorter
    // rounds; at order 129 also a lane's share of a column pair that fits in
    // registers)
    typedef JacobiShape<NMAX, (KC == 32 || KC == 64 || KC == 128) ? 8 : 4> J;
};

// the FP32 cores of buckets up to 64 can take the secular path
template <int KC, bool WITH_J>
__host__ __device__ constexpr bool core_secular() { return !WITH_J && KC <= 64; }

// FP64 cores of the widest bucket keep the accumulated rotations J in global
// memory (Req::Jg): K and J of order 129 (2 x 133 KB) exceed the LDS
template <int KC, bool WITH_J>
__host__ __device__ constexpr bool core_j_global() { return WITH_J && KC > 64; }

// threads of a core block: the Jacobi shape's, or for the secular (FP32
// append) cores of every bucket kSecCoreThreads: four lanes per pole at order
// 65 (roots, weights, norms, sort and sign take one lane group per column),
// one launch for the cores of all those buckets, and two blocks of the
// widest bucket per compute unit (registers and LDS)
constexpr int kSecCoreThreads = 384;
template <int KC, bool WITH_J>
__host__ __device__ constexpr int core_nt() {
    return core_secular<KC, WITH_J>() ? kSecCoreThreads : CoreShape<KC>::J::NT;
}

// Column stride (doubles) of the core's matrices in LDS: the Jacobi shape's,
// or for the secular cores the order rounded up to even (their Jacobi
// fallback then guards its rows), which keeps the widest one within half of
// a compute unit's LDS so that two cores share it.
template <int KC, bool WITH_J>
__host__ __device__ constexpr int core_ldw() {
    return core_secular<KC, WITH_J>() ? CoreShape<KC>::NMAX + (CoreShape<KC>::NMAX & 1) : CoreShape<KC>::J::LDW;
}

// Row stride (doubles) of W and W^-1 staged in LDS for the deferred-U
// products: KC + 2 spreads the rows of a 16-row operand over the banks.
template <int KC>
__host__ __device__ constexpr int core_wst() { return KC + 2; }

// dynamic LDS (doubles) of a core block of bucket KC; the secular (FP32
// append) cores stage A^T in the V_K region and W, then W^-1, in the K V one
template <int KC, bool WITH_J>
__host__ __device__ constexpr size_t core_lds_base() {
    constexpr bool SEC = core_secular<KC, WITH_J>();
    constexpr bool JLDS = (WITH_J && !core_j_global<KC, WITH_J>()) || SEC;
    return (size_t)(JLDS ? 2 : 1) * CoreShape<KC>::NMAX * core_ldw<KC, WITH_J>() +
           (size_t)8 * CoreShape<KC>::NMAX +
           (size_t)(SEC ? secular_scratch_doubles(CoreShape<KC>::NMAX) : 0);
}
template <int KC, bool WITH_J>
__host__ __device__ constexpr size_t core_lds_doubles() {
    static_assert(KC * core_wst<KC>() <= CoreShape<KC>::NMAX * core_ldw<KC, WITH_J>(), "A^T, W fit a matrix region");
    // (+1: room to align the region to 16 bytes)
    return core_lds_base<KC, WITH_J>() + 1;
}
// global doubles of Req::Jg for a stream of bucket KC
__host__ __device__ constexpr size_t core_jg_doubles(int KC) {
    return KC > 64 ? (size_t)CoreShape<128>::NMAX * CoreShape<128>::J::LDW : 0;
}

// The core of one request, one block (core_nt<KC, T == double>() threads,
// core_lds_doubles<KC, ...>() doubles of dynamic LDS).
template <typename T, int KC>
__device__ __attribute__((always_inline)) inline void core_block(const Req* __restrict__ rqp) {
    const Req& rq = *rqp;
    constexpr bool WITH_J = sizeof(T) == 8;
    constexpr bool SEC = core_secular<KC, WITH_J>();
    constexpr bool JG = core_j_global<KC, WITH_J>();
    // the dynamic region starts where the static one ends, 8-byte aligned;
    // the deferred-U products move pairs of doubles, which need 16 bytes
    extern __shared__ double smem_raw[];
    double* smem = smem_raw + (((uintptr_t)smem_raw & 15) ? 1 : 0);
    __shared__ double s_sc[8];
    __shared__ int s_i[4];
    __shared__ int s_sec[4];
    ISVD_GLOBAL DevHeader* hdr = gmem(rq.hdr);
    ISVD_GLOBAL ReqScratch* rs = gmem(rq.rs);
    const int k = hdr->k, ld = hdr->ld, cur = hdr->cur;
    const int kind = rq.kind;
    const int N = kind == kEntry ? k : k + 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int ldw = core_ldw<KC, WITH_J>();
    double* W = smem;
    // V_K: WITH_J (in global memory for the widest FP64 cores), or the secular path
    // regions at fixed offsets (the bucket's largest order), so that each
    // matrix region holds a KC x KC operand of the deferred-U products
    constexpr size_t MREG = (size_t)CoreShape<KC>::NMAX * core_ldw<KC, WITH_J>();
    double* J = JG ? rq.Jg : W + MREG;
    double* sS = W + MREG + (((WITH_J && !JG) || SEC) ? MREG : 0); // Sigma (k)
    double* sp = sS + N;                           // p (row / column) or s_v (rank-1)
    double* sig = sp + N;
    double* sgn = sig + N;
    double* tmp = sgn + N;
    int* perm = (int*)(tmp + N);
    double* su = tmp + 2 * N;                      // s_u (rank-1, no J); then sgn_j / sigma_j
    double* dcol = su + N;                         // s_u . W[:, c] (rank-1, no J)
    double* xsec = dcol + N;                       // secular scratch

    // projection sums of an append: the k_proj partials added in block order
    const size_t total = core_lds_doubles<KC, WITH_J>() - 1;   // past the alignment slack
    double* src1 = smem + total - 2 * (KC + 2);
    double* src2 = src1 + (KC + 2);
    if (kind != kEntry) {
        for (int c = tid; c < 2 * (KC + 2); c += nt) {
            const int cc = c < KC + 2 ? c : c - (KC + 2);
            const ISVD_GLOBAL double* part = gmem(c < KC + 2 ? rq.partials : rq.partials2);
            double s1 = 0.0;
            if (cc < k || cc >= KC)
                for (int t = 0; t < rq.proj_tiles; ++t) s1 += part[(size_t)t * (KC + 2) + cc];
            (c < KC + 2 ? src1 : src2)[cc] = s1;
        }
        __syncthreads();
    }
    double pc = 0.0;
    if (kind != kEntry && tid < k) pc = src1[tid] + src2[tid];
    // ||p2||^2, reduced by wave 0
    double p2sq = 0.0;
    if (kind != kEntry && tid < 64) {
        for (int c = tid; c < k; c += 64) p2sq += src2[c] * src2[c];
        for (int o = 32; o > 0; o >>= 1) p2sq += __shfl_xor(p2sq, o);
    }
    if (tid == 0) {
        int skip = hdr->status != 0 ? 1 : 0;
        double rho = 0.0, xnorm = 0.0, inv_rho = 0.0;
        int newdir = 0;
        if (kind != kEntry) {
            if (src1[KC + 1] > 0.0) skip = 1;
            const double z1sq = src2[KC];
            const double ysq = src1[KC];
            const double r2 = z1sq - p2sq;
            rho = r2 > 0.0 ? sqrt(r2) : 0.0;
            xnorm = sqrt(ysq);
            newdir = rho > rq.tol_rel * xnorm ? 1 : 0;
            if (!newdir) rho = 0.0;
            inv_rho = newdir ? 1.0 / rho : 0.0;
            if (!isfinite(rho) || !isfinite(xnorm)) skip = 1;
        } else {
            if (!isfinite(rq.delta)) skip = 1;
        }
        s_i[0] = skip;
        s_i[1] = newdir;
        s_sc[0] = rho;
        s_sc[1] = xnorm;
        s_sc[2] = inv_rho;
        s_sc[3] = kind != kEntry ? src1[KC] : 0.0;
    }
    __syncthreads();
    if (s_i[0]) {
        if (tid == 0) {
            rs->skip = 1;
            if (hdr->status == 0) hdr->status = -4;
            hdr->n_rejected += 1;
        }
        return;
    }
    const double rho = s_sc[0];
    // p = p1 + p2 (also kept in global memory for the rotation, which recomputes z^ per row)
    for (int c = tid; c < k; c += nt) {
        sS[c] = gmem(rq.S)[c];
        if (kind != kEntry) {
            sp[c] = pc;
            gmem(rq.p)[c] = pc;
        } else {
            if constexpr (!WITH_J) su[c] = (double)gmem((const T*)rq.U[cur])[uvo(rq.i, c, ld)];
            sp[c] = (double)gmem((const T*)rq.V[cur])[uvo(rq.j, c, ld)];
        }
    }
    __syncthreads();
    // assemble K (column-major in W, zero padding rows) and J = I
    for (int e = tid; e < N * ldw; e += nt) {
        const int col = e / ldw, row = e % ldw;
        double v = 0.0;
        if (row >= N) {
            W[e] = 0.0;
            if constexpr (WITH_J) J[e] = 0.0;
            continue;
        }
        if (kind == kEntry) {
            const double uu = WITH_J ? (double)gmem((const T*)rq.U[cur])[uvo(rq.i, row, ld)] : su[row];
            v = (row == col ? sS[row] : 0.0) + rq.delta * uu * sp[col];
        } else {
            if (row < k) v = (row == col) ? sS[row] : 0.0;
            else v = (col < k) ? sp[col] : rho;
        }
        W[e] = v;
        if constexpr (WITH_J) J[e] = (row == col) ? 1.0 : 0.0;
    }
    __syncthreads();
    bool use_sec = false;
    if constexpr (SEC) {
        if (kind != kEntry) use_sec = secular_append_core<CoreShape<KC>::NMAX, core_nt<KC, WITH_J>()>(sS, sp, rho, k, rq.k_keep < N ? rq.k_keep : N, W, J, ldw,
                                                          xsec, s_sec);
    }
    // FP32 storage rounds U_K, V_K to 6e-8: columns orthogonal to 1e-10 suffice
    const int sweeps = use_sec ? 0
                               : jacobi_block<CoreShape<KC>::NMAX, WITH_J, CoreShape<KC>::J::TPP, SEC>(
                                     W, J, N, ldw, 40, WITH_J ? 0.0 : 1e-10);
    constexpr int NTC = core_nt<KC, WITH_J>();
    // a deferred-U stream's W and W^-1 (current parity, KC x KC each): the
    // loads are issued here and complete during the sort, the signs and the
    // rotation outputs; they are staged in LDS for the products
    constexpr int PF = SEC ? (KC * KC + NTC - 1) / NTC : 1;   // pairs of doubles of both matrices per thread
    gvec_d2 pf[PF];
    if constexpr (SEC) {
        if (kind == kRow && rq.Wd[0] != nullptr) {
            const int wp0 = hdr->wpar;
            const ISVD_GLOBAL gvec_d2* w2 = gmem((const gvec_d2*)rq.Wd[wp0]);
            const ISVD_GLOBAL gvec_d2* wi2 = gmem((const gvec_d2*)rq.Wdi[wp0]);
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int e = tid + q * NTC;   // [0, KC^2 / 2): W, then W^-1
                if (e < KC * KC / 2) pf[q] = w2[e];
                else if (e < KC * KC) pf[q] = wi2[e - KC * KC / 2];
            }
        }
    }
    // singular values: the column norms of W, one GS-lane group per column,
    // sorted non-increasing (ties: lower column first)
    constexpr int GS = sec_lanes(CoreShape<KC>::NMAX, NTC);
    const int gs = tid / GS, ls = tid % GS;
    for (int c = gs; c < N; c += NTC / GS) {
        const double* w = W + (size_t)c * ldw;
        double s2 = 0.0;
        for (int e = ls; e < N; e += GS) s2 += w[e] * w[e];
        s2 = dpp_group_sum<GS>(s2);
        if (ls == 0) tmp[c] = sqrt(s2);
    }
    __syncthreads();
    for (int c = gs; c < N; c += NTC / GS) {
        const double sc = tmp[c];
        double r = 0.0;
        for (int d = ls; d < N; d += GS) {
            const double sd = tmp[d];
            r += (sd > sc || (sd == sc && d < c)) ? 1.0 : 0.0;
        }
        r = dpp_group_sum<GS>(r);
        if (ls == 0) {
            perm[(int)r] = c;
            sig[(int)r] = sc;
        }
    }
    __syncthreads();
    if constexpr (!WITH_J) {
        if (kind == kEntry) {
            for (int c = tid; c < N; c += nt) {
                double d = 0.0;
                for (int i = 0; i < N; ++i) d += su[i] * W[(size_t)c * ldw + i];
                dcol[c] = d;
            }
            __syncthreads();
        }
    }
    // right singular vector entry e of column c of W (unsorted, unsigned)
    auto vraw = [&](int e, int c) -> double {
        if constexpr (WITH_J) {
            return J[(size_t)c * ldw + e];
        } else {
            if (use_sec) return J[(size_t)c * ldw + e];
            const double* w = W + (size_t)c * ldw;
            const double s2 = tmp[c] * tmp[c];
            if (!(s2 > 0.0)) return 0.0;
            double kw;
            if (kind == kEntry) kw = sS[e] * w[e] + rq.delta * sp[e] * dcol[c];
            else if (e < k) kw = sS[e] * w[e] + sp[e] * w[k];
            else kw = rho * w[k];
            return kw / s2;
        }
    };
    // signs: the largest-magnitude entry of each right vector positive (the
    // first one on ties), one GS-lane group per vector
    for (int jj = gs; jj < N; jj += NTC / GS) {
        const int c = perm[jj];
        int imax = N;
        double vmax = -1.0;
        for (int e = ls; e < N; e += GS) {
            const double a = fabs(vraw(e, c));
            if (a > vmax) {
                vmax = a;
                imax = e;
            }
        }
        dpp_group_argmax<GS>(vmax, imax);
        if (imax >= N) imax = 0;
        if (ls == 0) sgn[jj] = vraw(imax, c) < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();
    int kout;
    if (kind == kEntry) {
        kout = k;
    } else {
        kout = rq.k_keep < N ? rq.k_keep : N;
        while (kout > 0 && sig[kout - 1] == 0.0) --kout;
    }
    const int ldo = round4(kout);
    // Drift signals (Sections 3.2-3.3): U_K, V_K have orthonormal columns, so the
    // cosines of the principal angles between the previous span (zero-padded)
    // and the new one are the singular values of the rotation's first k rows,
    // and for kout <= k the smallest is sqrt(1 - |last row|^2).  A grown rank
    // contains the previous span; a rank-one update keeps both spans.  For a
    // column append U's rotation is V_K and V's is U_K.  Wave 0 reduces; tid 0
    // keeps the squared sines.
    double sin2_u = 0.0, sin2_v = 0.0;
    if (kind != kEntry && kout <= k && tid < 64) {
        double bu = 0.0, bv = 0.0;
        for (int j = tid; j < kout; j += 64) {
            const int c = perm[j];
            const double uk = sig[j] > 0.0 ? W[(size_t)c * ldw + k] / sig[j] : 0.0;
            const double vk = vraw(k, c);
            bu += uk * uk;
            bv += vk * vk;
        }
        for (int o = 32; o > 0; o >>= 1) {
            bu += __shfl_xor(bu, o);
            bv += __shfl_xor(bv, o);
        }
        sin2_u = kind == kRow ? bu : bv;
        sin2_v = kind == kRow ? bv : bu;
    }
    ISVD_GLOBAL T* QU = gmem((T*)rq.QU);
    ISVD_GLOBAL T* QV = gmem((T*)rq.QV);
    // Deferred U (U = U0 W, Brand): a row append whose rank stays k and whose
    // new row b = U_K[k, :k] has |b|^2 <= 1/2 is applied to W alone when the
    // host asks for it; otherwise W is folded into the rotation of U.
    bool wd = false, defer = false;
    if constexpr (!WITH_J) {
        wd = kind == kRow && rq.Wd[0] != nullptr;
        if (wd) {
            if (tid == 0) {
                const double bb = sin2_u;   // |b|^2: the last row of U_K, reduced by wave 0 above
                s_i[2] = (rq.defer && kout == k && ldo == ld && bb <= 0.5) ? 1 : 0;
                s_sc[4] = bb;
            }
            __syncthreads();
            defer = s_i[2] != 0;
        }
    }
    // U_K(e, j) = sgn_j W[e, perm_j] / sigma_j ;  V_K(e, j) = sgn_j vraw(e, perm_j)
    double* fsg = su;   // sgn_j / sigma_j (s_u is no longer needed)
    for (int j = tid; j < kout; j += nt) fsg[j] = sig[j] > 0.0 ? sgn[j] / sig[j] : 0.0;
    __syncthreads();
    for (int e = tid; e < N * ldo; e += nt) {
        const int row = e / ldo, j = e % ldo;
        double uk = 0.0, vk = 0.0;
        if (j < kout) {
            const int c = perm[j];
            uk = fsg[j] * W[(size_t)c * ldw + row];
            vk = sgn[j] * vraw(row, c);
        }
        if (kind == kEntry) {
            QU[e] = (T)uk;
            QV[e] = (T)vk;
        } else if (kind == kRow) {
            if (row < k) {
                if (!wd) QU[e] = (T)uk;   // with W, QU is W A (explicit) or unused (deferred)
            }
            else if (!defer) gmem((T*)rq.U[cur ^ 1])[uvo(rq.m, j, ldo)] = (T)uk;
            QV[e] = (T)vk;
        } else {
            QU[e] = (T)vk;
            if (row < k) QV[e] = (T)uk;
            else gmem((T*)rq.V[cur ^ 1])[uvo(rq.n, j, ldo)] = (T)uk;
        }
    }
    for (int j = tid; j < kout; j += nt) gmem(rq.S)[j] = sig[j];
    if constexpr (SEC) {
        if (wd) {
            // W, W^-1: KC x KC row-major (entries past k are never read).  With
            // A = U_K[0:k, 0:k], b = U_K[k, 0:k] (A^T A + b^T b = I) and
            // f_j = sgn_j / sigma_j: A[c][j] = f_j Kv[perm_j][c], b_j =
            // f_j Kv[perm_j][k] (Kv: the columns of K V in LDS).
            //   deferred: W' = W A and W'^-1 = A^-1 W^-1 with A^-1 =
            //     (I + b^T b / (1 - |b|^2)) A^T, i.e. A^-1[r][c] = A[c][r] +
            //     b_r v_c for v = b A^T / (1 - |b|^2); the new row of U0 is
            //     u0 = b W'^-1 = v W^-1.
            //   explicit: U's rotation takes W A, and W, W^-1 return to I.
            // The products run on the FP64 matrix cores
            // (v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16] and
            // B[l/16][l%16]; D[4r + l/16][l%16] is the lane's r-th value), one
            // 16 x 16 output tile per wave at a time (at most four waves, one
            // per SIMD); lane quarter q takes the contraction indices
            // [q KC/4, (q+1) KC/4), so each lane reads its operands from LDS
            // as contiguous runs: rows of W, of W^-1's transpose, and of A^T,
            // first gathered from K V in sorted order.
            const int wp = hdr->wpar;
            double* bv = xsec;                                  // b (k)
            double* gv = xsec + CoreShape<KC>::NMAX;            // f_j b_j (k)
            double* vv = xsec + 2 * CoreShape<KC>::NMAX;        // v (k)
            constexpr int WST = core_wst<KC>();
            static_assert(core_lds_base<KC, WITH_J>() % 2 == 0 && WST % 2 == 0 && core_ldw<KC, WITH_J>() % 2 == 0,
                          "16-byte rows");
            double* At = J;        // A^T (the V_K region is free once the outputs are written)
            double* Wst = W;       // W, then W^-1 transposed (the K V region, once A^T and v are formed)
            __syncthreads();
            for (int j = tid; j < kout; j += nt) {
                const double f = sgn[j] / sig[j];
                const double kb = W[(size_t)perm[j] * ldw + k];
                sgn[j] = f;
                bv[j] = f * kb;
                gv[j] = f * f * kb;
            }
            __syncthreads();
            // A^T[j][c] = f_j Kv[perm_j][c] for j < kout, c < k; zero elsewhere in KC x KC
            for (int e = tid; e < KC * KC; e += nt) {
                const int j = e / KC, c = e % KC;
                At[j * WST + c] = (j < kout && c < k) ? sgn[j] * W[(size_t)perm[j] * ldw + c] : 0.0;
            }
            if (defer) {
                // v (zero past k) and b (zero past k)
                const double ib = 1.0 / (1.0 - s_sc[4]);
                for (int c = gs; c < KC; c += NTC / GS) {
                    double a = 0.0;
                    if (c < k)
                        for (int j = ls; j < k; j += GS) a += gv[j] * W[(size_t)perm[j] * ldw + c];
                    a = dpp_group_sum<GS>(a);
                    if (ls == 0) vv[c] = a * ib;
                }
                for (int j = k + tid; j < KC; j += nt) bv[j] = 0.0;
            } else {
                for (int c = tid; c < KC; c += nt) {
                    vv[c] = 0.0;
                    bv[c] = 0.0;
                }
            }
            __syncthreads();
            // stage one of the prefetched matrices (entries outside the leading
            // k x k block as zeros, so the products need no masks): W row-major,
            // or W^-1 transposed
            auto stage = [&](bool inverse) {
#pragma unroll
                for (int q = 0; q < PF; ++q) {
                    const int e = tid + q * NTC;
                    if (!inverse && e < KC * KC / 2) {
                        const int r = 2 * e / KC, c = 2 * e % KC;
                        gvec_d2 v = pf[q];
                        v.x = (r < k && c < k) ? v.x : 0.0;
                        v.y = (r < k && c + 1 < k) ? v.y : 0.0;
                        *(gvec_d2*)(Wst + r * WST + c) = v;
                    } else if (inverse && e >= KC * KC / 2 && e < KC * KC) {
                        const int e2 = 2 * (e - KC * KC / 2), r = e2 / KC, c = e2 % KC;
                        Wst[c * WST + r] = (r < k && c < k) ? pf[q].x : 0.0;
                        Wst[(c + 1) * WST + r] = (r < k && c + 1 < k) ? pf[q].y : 0.0;
                    }
                }
            };
            stage(false);
            __syncthreads();
            constexpr int S = KC / 4;
            const int lane = tid & 63, wave = tid >> 6;
            const int twv = (nt >> 6) < 4 ? (nt >> 6) : 4;     // waves on the products (one per SIMD)
            const int li = lane & 15, lq = lane >> 4;
            const int c0 = lq * S;
            const int kt = (k + 15) / 16;
            const int jt = defer ? kt : (ldo + 15) / 16;
            ISVD_GLOBAL double* Wn = gmem(rq.Wd[wp ^ 1]);
            ISVD_GLOBAL double* Win = gmem(rq.Wdi[wp ^ 1]);
            ISVD_GLOBAL T* U0 = gmem((T*)rq.U[cur]);
            // inv = 0: W A (or, explicit, U's rotation); inv = 1: A^-1 W^-1 and u0
            for (int inv = 0; inv < (defer ? 2 : 1); ++inv) {
                if (inv) {
                    __syncthreads();   // every read of W is done
                    stage(true);
                    __syncthreads();
                }
                for (int t = wave; t < kt * jt && wave < twv; t += twv) {
                    const int r0 = (t / jt) * 16, j0 = (t % jt) * 16;
                    const int ra = r0 + li, jb = j0 + li;
                    double av[S], bw[S];
                    // operand rows past k (or past k_out) are zero in LDS
                    const double2* pa;
                    const double2* pb;
                    double br = 0.0;
                    if (!inv) {
                        pa = (const double2*)(Wst + ra * WST + c0);   // row ra of W
                        pb = (const double2*)(At + jb * WST + c0);    // column jb of A (row jb of A^T)
                    } else {
                        pa = (const double2*)(At + ra * WST + c0);    // row ra of A^-1 = A^T + b^T v ...
                        pb = (const double2*)(Wst + jb * WST + c0);   // column jb of W^-1 (a row of its transpose)
                        br = bv[ra];
                    }
                    const double2* vp = (const double2*)(vv + c0);    // ... + b_ra v
#pragma unroll
                    for (int s2 = 0; s2 < S / 2; ++s2) {
                        const double2 x = pa[s2], y = pb[s2], z = vp[s2];
                        av[2 * s2] = x.x + br * z.x;
                        av[2 * s2 + 1] = x.y + br * z.y;
                        bw[2 * s2] = y.x;
                        bw[2 * s2 + 1] = y.y;
                    }
                    core_v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int q = 0; q < S; ++q)
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bw[q], acc, 0, 0, 0);
                    if (!defer) {
                        for (int r = 0; r < 4; ++r) {
                            const int row = r0 + 4 * r + lq;
                            if (row < k && jb < ldo) QU[row * ldo + jb] = (T)acc[r];
                        }
                    } else {
                        ISVD_GLOBAL double* out = inv ? Win : Wn;
                        for (int r = 0; r < 4; ++r) {
                            const int row = r0 + 4 * r + lq;
                            if (row < k && jb < k) out[(size_t)row * KC + jb] = acc[r];
                        }
                        if (inv && r0 == 0) {
                            // u0[jb] = v W^-1[:, jb]: this lane's contraction indices, then the four quarters
                            double up = 0.0;
#pragma unroll
                            for (int q = 0; q < S; ++q) up += vv[c0 + q] * bw[q];
                            up += __shfl_xor(up, 16);
                            up += __shfl_xor(up, 32);
                            if (lq == 0 && jb < ld) U0[uvo(rq.m, jb, ld)] = (T)(jb < k ? up : 0.0);
                        }
                    }
                }
            }
            if (!defer) {
                __syncthreads();
                for (int e = tid; e < KC * KC; e += nt) {
                    const double v = (e / KC == e - (e / KC) * KC) ? 1.0 : 0.0;
                    gmem(rq.Wd[wp])[e] = v;
                    gmem(rq.Wdi[wp])[e] = v;
                }
            }
        }
    }
    // sums over the kept / previous spectrum, reduced by wave 0
    double s2 = 0.0, ds = 0.0, so = 0.0;
    if (tid < 64) {
        const int kmax = kout > k ? kout : k;
        for (int j = tid; j < kmax; j += 64) {
            const double sn = j < kout ? sig[j] : 0.0, sv = j < k ? sS[j] : 0.0;
            s2 += sn * sn;
            ds += (sn - sv) * (sn - sv);
            so += sv * sv;
        }
        for (int o = 32; o > 0; o >>= 1) {
            s2 += __shfl_xor(s2, o);
            ds += __shfl_xor(ds, o);
            so += __shfl_xor(so, o);
        }
    }
    if (tid == 0) {
        double dN = 0.0;
        if (kind == kEntry) {
            ISVD_GLOBAL T* A = gmem((T*)rq.A);
            const double aold = (double)A[rq.i * rq.lda + rq.j];
            A[rq.i * rq.lda + rq.j] = (T)(aold + rq.delta);
            dN = 2.0 * rq.delta * aold + rq.delta * rq.delta;
        } else {
            dN = s_sc[3];
        }
        rs->skip = 0;
        rs->k_in = k;
        rs->ld_in = ld;
        rs->k_out = kout;
        rs->ld_out = ldo;
        rs->in_idx = cur;
        rs->inv_rho = s_sc[2];
        rs->deferred = defer ? 1 : 0;
        hdr->k = kout;
        hdr->ld = ldo;
        hdr->cur = defer ? cur : (cur ^ 1);
        if (defer) hdr->wpar ^= 1;
        hdr->t += 1;
        if (kind == kRow) hdr->m += 1;
        if (kind == kCol) hdr->n += 1;
        hdr->N += dN;
        hdr->sweeps = sweeps;
        hdr->last_kind = kind;
        hdr->sigma2 = s2;
        hdr->step_angle_u = asin(sqrt(fmin(sin2_u, 1.0)));
        hdr->step_angle_v = asin(sqrt(fmin(sin2_v, 1.0)));
        hdr->spec_change = so > 0.0 ? sqrt(ds / so) : __builtin_nan("");
        hdr->sigma_last = kout > 0 ? sig[kout - 1] : 0.0;
        if (kind != kEntry) {
            hdr->rho = rho;
            hdr->xnorm = s_sc[1];
            hdr->novelty = s_sc[1] > 0.0 ? rho / s_sc[1] : 0.0;
            hdr->new_dir = s_i[1];
            hdr->sigma_dropped = kout < N ? sig[kout] : 0.0;
        }
    }
}

template <typename T, int KC>
__global__ void __launch_bounds__((core_nt<KC, sizeof(T) == 8>())) k_core(const Req* __restrict__ reqs) {
    core_block<T, KC>(reqs + blockIdx.x);
}

// ---------------------------------------------------------------------------
// Rotation (the "update singular vectors" step): X'[r, :] = X[r, 0:k] Q[0:k, :]
// (+ z^_r Q[k, :] for the projected basis of an append, with
// z^_r = (y_r - X[r, :] p) / rho), written out-of-place into the other buffer
// with the new leading dimension.  The projected basis' tiles also write the
// payload into A (row m of A for a row append, column n for a column append).
// Generic VALU version: block = rot_rows(KC) rows of one basis of one request.
// Every rotation kernel takes `part`: 0 = the tiles of U then V of each
// request, 1 = U's tiles only, 2 = V's tiles only (prefix over those tiles).
template <typename T, int KC>
__global__ void __launch_bounds__(kThreads) k_rotate(const Req* __restrict__ reqs,
                                                     const int* __restrict__ prefix, int nreq, int part) {
    constexpr int RT = rot_rows(KC);
    __shared__ T sQ[(KC + 1) * KC];
    __shared__ T sX[RT * KC];
    __shared__ double sz[RT];
    __shared__ double sp[KC];
    // a grid sized for more tiles than this launch has (a captured tick,
    // sized for the streams' capacity) leaves the extra blocks idle
    if ((int)blockIdx.x >= prefix[nreq]) return;
    const int ri = find_req(prefix, nreq, blockIdx.x);
    const Req& rq = reqs[ri];
    const ReqScratch* rs = rq.rs;
    if (rs->skip) return;
    const int tile_all = blockIdx.x - prefix[ri];
    const bool isU = part == 1 || (part == 0 && tile_all < rq.rot_tiles_u);
    const int tile = (part != 0 || isU) ? tile_all : tile_all - rq.rot_tiles_u;
    const bool deferred = rs->deferred != 0;   // deferred U: see k_rotate_mfma_t
    if (isU && deferred) return;
    const int kin = rs->k_in, ldi = rs->ld_in, ldo = rs->ld_out, idx = rs->in_idx;
    const int64_t rows = isU ? rq.m : rq.n;
    const T* Xi = (const T*)(isU ? rq.U[idx] : rq.V[idx]);
    T* Xo = (T*)(isU ? rq.U[idx ^ 1] : rq.V[deferred ? idx : idx ^ 1]);
    const T* Q = (const T*)(isU ? rq.QU : rq.QV);
    const bool projected = (rq.kind == kRow && !isU) || (rq.kind == kCol && isU);
    const int nq = kin + (projected ? 1 : 0);
    for (int e = threadIdx.x; e < nq * ldo; e += kThreads) sQ[e] = Q[e];
    const int64_t r0 = (int64_t)tile * RT;              // a multiple of 16: whole tiles
    const int nr = (int)min((int64_t)RT, rows - r0);
    const int ntl = (nr + 15) & ~15;                     // rows of the tiles loaded
    for (int e = threadIdx.x; e < ntl * ldi; e += kThreads) sX[e] = Xi[r0 * ldi + e];
    if (projected)
        for (int c = threadIdx.x; c < kin; c += kThreads) sp[c] = rq.p[c];
    __syncthreads();
    if (projected) {
        const T* y = (const T*)rq.payload;
        const double inv_rho = rs->inv_rho;
        T* A = (T*)rq.A;
        for (int rr = threadIdx.x; rr < nr; rr += kThreads) {
            double d = 0.0;
            for (int c = 0; c < kin; ++c) d += (double)sX[uvo(rr, c, ldi)] * sp[c];
            const T yv = y[r0 + rr];
            sz[rr] = ((double)yv - d) * inv_rho;
            if (rq.kind == kRow) A[rq.m * rq.lda + r0 + rr] = yv;
            else A[(r0 + rr) * rq.lda + rq.n] = yv;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * ldo; e += kThreads) {
        const int rr = e / ldo, j = e % ldo;
        T acc = (T)0;
        for (int c = 0; c < kin; ++c) acc += sX[uvo(rr, c, ldi)] * sQ[c * ldo + j];
        if (projected) acc += (T)sz[rr] * sQ[kin * ldo + j];
        Xo[uvo(r0 + rr, j, ldo)] = acc;
    }
}

// ---------------------------------------------------------------------------
// FP32 rotation on the matrix cores (v_mfma_f32_16x16x4f32): the same
// X' = X Q (+ z^ Q[k, :]) as k_rotate.  A wave works on 16-row tiles; a
// tile of U or V is contiguous in HBM (16 x ld floats), so it is loaded and
// stored with contiguous dwordx4 accesses (64 lanes x 16 B per instruction)
// and staged through LDS; the next tile's loads are issued before the
// current tile's MFMAs.  MFMA operands: lane l owns row l%16 and the
// contiguous k-range [g*S, g*S+S) (g = l/16, S = KC/4) of it, the MFMA's
// k order is permuted to match (step s feeds k = g*S + s of every lane
// group); Q sits in LDS in the same order.  Output lane layout of the
// 16x16x4 FP32 instruction: D[4*(l/16) + r][l%16].  FP32 accumulation.
typedef float mfma_v4f __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, rounded to nearest even (finite inputs)
__device__ inline short to_bf16(float f) {
    const unsigned u = __float_as_uint(f);
    return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
typedef __attribute__((address_space(1))) const float gcfloat;
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) const mfma_v4f gcf4;
typedef __attribute__((address_space(1))) mfma_v4f gf4;

template <int KC>
__global__ void __launch_bounds__(kThreads) k_rotate_mfma(const Req* __restrict__ reqs,
                                                          const int* __restrict__ prefix, int nreq, int part) {
    constexpr int S = KC / 4;                 // k-steps (and elements per lane)
    constexpr int NB = KC >= 16 ? KC / 16 : 1;
    constexpr int NCOL = NB * 16;             // output columns computed
    constexpr int XP = KC + 4;                // LDS row stride of X tiles (bank spread)
    constexpr int OP = NCOL + 4;              // LDS row stride of output tiles
    constexpr int QP = NCOL + 4;              // LDS row stride of Q
    constexpr int STEPS = kMfmaRotRows / (4 * 16);
    constexpr int VPL = (16 * KC / 4 + 63) / 64;   // float4 per lane per tile (upper bound)
    __shared__ float sQ[(KC + 1) * QP];
    __shared__ float sX[4][16 * XP];
    __shared__ float sO[4][16 * OP];
    __shared__ double sp[KC];
    // a grid sized for more tiles than this launch has (a captured tick,
    // sized for the streams' capacity) leaves the extra blocks idle
    if ((int)blockIdx.x >= prefix[nreq]) return;
    const int ri = find_req(prefix, nreq, blockIdx.x);
    const Req& rq = reqs[ri];
    const ReqScratch* rs = rq.rs;
    if (rs->skip) return;
    const int tile_all = blockIdx.x - prefix[ri];
    const bool isU = part == 1 || (part == 0 && tile_all < rq.rot_tiles_u);
    const int tile = (part != 0 || isU) ? tile_all : tile_all - rq.rot_tiles_u;
    // a row append applied to W (deferred U) rotates no U tile and V in
    // place (same leading dimension; each row is read before it is written,
    // by the same wave)
    const bool deferred = rs->deferred != 0;
    if (isU && deferred) return;
    const int kin = rs->k_in, ldi = rs->ld_in, ldo = rs->ld_out, idx = rs->in_idx;
    const int64_t rows = isU ? rq.m : rq.n;
    gcfloat* Xi = (gcfloat*)(isU ? rq.U[idx] : rq.V[idx]);
    gfloat* Xo = (gfloat*)(isU ? rq.U[idx ^ 1] : rq.V[deferred ? idx : idx ^ 1]);
    gcfloat* Q = (gcfloat*)(isU ? rq.QU : rq.QV);
    const bool projected = (rq.kind == kRow && !isU) || (rq.kind == kCol && isU);
    const int nq = kin + (projected ? 1 : 0);
    for (int e = threadIdx.x; e < (KC + 1) * QP; e += kThreads) {
        const int kk = e / QP, j = e % QP;
        sQ[e] = (kk < nq && j < ldo) ? Q[kk * ldo + j] : 0.0f;
    }
    if (projected)
        for (int c = threadIdx.x; c < KC; c += kThreads) sp[c] = c < kin ? rq.p[c] : 0.0;
    __syncthreads();
    const int l = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = l >> 4, col = l & 15;
    // B operand in registers for the narrow buckets; from LDS for the wide
    // ones, where registers for it would cost occupancy (measured slower)
    constexpr bool BREG = NB * S <= 16;
    float bq[BREG ? NB : 1][BREG ? S : 1];
    if constexpr (BREG) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int s4 = 0; s4 < S; ++s4) bq[nb][s4] = sQ[(g * S + s4) * QP + 16 * nb + col];
    }
    float* sx = sX[wave];
    float* so = sO[wave];
    const int64_t base = (int64_t)tile * kMfmaRotRows;
    const int ntile_vec_in = 4 * ldi;       // float4 per 16-row input tile
    const int ntile_vec_out = 4 * ldo;
    // prefetch of a tile into registers
    mfma_v4f pre[VPL];
    auto fetch = [&](int64_t row0, int nr) {
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            const int f = l + 64 * v;
            // a whole 16-row tile (contiguous); rows past the basis are not stored
            if (f < ntile_vec_in && nr > 0) pre[v] = ((gcf4*)(Xi + row0 * ldi))[f];
            else pre[v] = (mfma_v4f){0.f, 0.f, 0.f, 0.f};
        }
    };
    int64_t row0 = base + (int64_t)wave * 16;
    int nr = row0 < rows ? (int)min((int64_t)16, rows - row0) : 0;
    if (nr > 0) fetch(row0, nr);
    const float* yv_base = (const float*)rq.payload;
    const double inv_rho = rs->inv_rho;
    for (int st = 0; st < STEPS; ++st) {
        if (nr <= 0) break;
        // registers -> LDS tile (row stride XP), zero columns >= kin
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            const int f = l + 64 * v;
            if (f < ntile_vec_in) {
                int r, c;
                uv_tile_rc(4 * f, &r, &c);
                float* d = sx + r * XP + c;
                d[0] = c + 0 < kin ? pre[v][0] : 0.0f;
                d[1] = c + 1 < kin ? pre[v][1] : 0.0f;
                d[2] = c + 2 < kin ? pre[v][2] : 0.0f;
                d[3] = c + 3 < kin ? pre[v][3] : 0.0f;
            }
        }
        for (int c = ldi + l; c < KC; c += 64)          // columns beyond ld_in
            for (int r = 0; r < 16; ++r) sx[r * XP + c] = 0.0f;
        // next tile's loads in flight during this tile's MFMAs
        const int64_t nrow0 = row0 + 64;
        const int nnr = (st + 1 < STEPS && nrow0 < rows) ? (int)min((int64_t)16, rows - nrow0) : 0;
        if (nnr > 0) fetch(nrow0, nnr);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        float a[S];
#pragma unroll
        for (int s4 = 0; s4 < S; ++s4) a[s4] = sx[col * XP + g * S + s4];
        mfma_v4f acc[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = (mfma_v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s4 = 0; s4 < S; ++s4)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                float bv;
                if constexpr (BREG) bv = bq[nb][s4];
                else bv = sQ[(g * S + s4) * QP + 16 * nb + col];
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s4], bv, acc[nb], 0, 0, 0);
            }
        if (projected) {
            // z^ of this lane's row (row l%16 of the tile), spread to the output layout
            double d = 0.0;
#pragma unroll
            for (int s4 = 0; s4 < S; ++s4) d += (double)a[s4] * sp[g * S + s4];
            d += __shfl_xor(d, 16);
            d += __shfl_xor(d, 32);
            const bool live = col < nr;
            const float yv = live ? yv_base[row0 + col] : 0.0f;
            const float z = (float)(((double)yv - d) * inv_rho);
            if (live && g == 0) {
                gfloat* A = (gfloat*)rq.A;
                if (rq.kind == kRow) A[rq.m * rq.lda + row0 + col] = yv;
                else A[(row0 + col) * rq.lda + rq.n] = yv;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float zj = __shfl(z, 4 * g + j);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[nb][j] += zj * sQ[kin * QP + 16 * nb + col];
            }
        }
        // accumulators -> LDS output tile -> contiguous stores
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int j = 0; j < 4; ++j) so[(4 * g + j) * OP + 16 * nb + col] = acc[nb][j];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        for (int f = l; f < ntile_vec_out; f += 64) {
            int r, c;
            uv_tile_rc(4 * f, &r, &c);
            if (r >= nr) continue;
            const float* src = so + r * OP + c;
            ((gf4*)(Xo + row0 * ldo))[f] = (mfma_v4f){src[0], src[1], src[2], src[3]};
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        row0 = nrow0;
        nr = nnr;
    }
}

// ---------------------------------------------------------------------------
// FP32 rotation on the matrix cores, transposed: X'^T = Q^T X^T with
// v_mfma_f32_16x16x4f32 (lane l: A[l%16][l/16], B[l/16][l%16],
// D[4(l/16)+r][l%16]).  Q^T is the A operand and stays in registers for all
// of a wave's row tiles.  X is the B operand: with the tiled basis layout,
// the q-th 16-column panel of a 16-row tile is 256 contiguous floats and
// lane l takes one float4 of it -- row l%16, columns 16 q + 4 (l/16) + 0..3 --
// so each load instruction reads 1 KB contiguous; the MFMA k order follows
// (step s: k = 16 (s/4) + 4 (l/16) + s%4).  The accumulators hold, for row
// l%16, the four output columns 16 nb + 4 (l/16) + r, which is again one
// float4 of the output tile's panel nb: stores are 1 KB contiguous too.  No
// LDS staging.  ROWS rows per block; a wave takes RT consecutive 16-row tiles
// per step (RT independent accumulator sets); with PF the next step's loads
// are issued before the current step's MFMAs.
// BF16: the products on the BF16 matrix cores (v_mfma_f32_16x16x16bf16_1k,
// operands rounded to nearest BF16, FP32 accumulation): lane l holds the 4
// k values 16 q + 4 (l/16) + 0..3 of a panel, which is exactly that
// instruction's operand layout, so one MFMA covers a whole panel.
// One block of rows (tile_all-th of the request, counted over U then V when
// part = 0) of one request.
template <int KC, int ROWS, int RT, bool PF, bool BF16 = false>
__device__ __attribute__((always_inline)) inline void rotate_mfma_t_block(const Req* __restrict__ rqp, int tile_all, int part) {
    const Req& rq = *rqp;
    constexpr int NQ = (KC + 15) / 16;           // panels (loads per lane per tile)
    constexpr int STEPS = 4 * NQ;                // MFMA k-steps per output block
    constexpr int NB = NQ;                       // 16-column output blocks
    constexpr int SROWS = 64 * RT;               // rows per block step (4 waves)
    constexpr int TSTEPS = ROWS / SROWS;
    __shared__ double sp[16 * NQ];
    __shared__ float sqz[16 * NB];
    const ISVD_GLOBAL ReqScratch* rs = gmem(rq.rs);
    if (rs->skip) return;
    const bool isU = part == 1 || (part == 0 && tile_all < rq.rot_tiles_u);
    const int tile = (part != 0 || isU) ? tile_all : tile_all - rq.rot_tiles_u;
    // a row append applied to W (deferred U) rotates no U tile and V in
    // place (same leading dimension; each row is read before it is written,
    // by the same wave)
    const bool deferred = rs->deferred != 0;
    if (isU && deferred) return;
    const int kin = rs->k_in, ldi = rs->ld_in, ldo = rs->ld_out, idx = rs->in_idx;
    const int64_t rows = isU ? rq.m : rq.n;
    gcfloat* Xi = (gcfloat*)(isU ? rq.U[idx] : rq.V[idx]);
    gfloat* Xo = (gfloat*)(isU ? rq.U[idx ^ 1] : rq.V[deferred ? idx : idx ^ 1]);
    gcfloat* Q = (gcfloat*)(isU ? rq.QU : rq.QV);
    const bool projected = (rq.kind == kRow && !isU) || (rq.kind == kCol && isU);
    if (projected) {
        for (int c = threadIdx.x; c < 16 * NQ; c += kThreads) sp[c] = c < kin ? gmem(rq.p)[c] : 0.0;
        for (int c = threadIdx.x; c < 16 * NB; c += kThreads) sqz[c] = c < ldo ? Q[kin * ldo + c] : 0.0f;
    }
    const int l = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = l >> 4, n = l & 15;
    // Q^T in registers: qa[nb][s] = Q[k(s)][16 nb + n]
    float qa[NB][BF16 ? 1 : STEPS];
    bf16x4 qb[NB][BF16 ? NQ : 1];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int s4 = 0; s4 < STEPS; ++s4) {
            const int k = 16 * (s4 >> 2) + 4 * g + (s4 & 3);
            const int c = 16 * nb + n;
            const float v = (k < kin && c < ldo) ? Q[k * ldo + c] : 0.0f;
            if constexpr (BF16) qb[nb][s4 >> 2][s4 & 3] = to_bf16(v);
            else qa[nb][s4] = v;
        }
    __syncthreads();
    mfma_v4f b[RT][NQ], bn[PF ? RT : 1][NQ];
    float yb[RT], ybn[PF ? RT : 1];
    const ISVD_GLOBAL float* yv_base = gmem((const float*)rq.payload);
    // the B operand of a step's tiles: panel q, 4-column group g, row n (zero
    // past the basis' rows or columns), and for the projected basis the
    // payload entry of row n, fetched with it
    auto fetch = [&](int64_t s0, mfma_v4f (*dst)[NQ], float* ydst) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t t0 = s0 + 16 * rt;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (t0 + n < rows && 16 * q + 4 * g < ldi)
                    dst[rt][q] = *(gcf4*)(Xi + t0 * ldi + 256 * q + 64 * g + 4 * n);
                else
                    dst[rt][q] = (mfma_v4f){0.f, 0.f, 0.f, 0.f};
            }
            ydst[rt] = (projected && t0 + n < rows) ? yv_base[t0 + n] : 0.0f;
        }
    };
    const double inv_rho = rs->inv_rho;
    int64_t row0 = (int64_t)tile * ROWS + wave * 16 * RT;
    fetch(row0, b, yb);
#pragma unroll 1
    for (int t = 0; t < TSTEPS; ++t) {
        if (row0 >= rows) break;
        const int64_t nrow0 = row0 + SROWS;
        if constexpr (PF) {
            if (t + 1 < TSTEPS) fetch(nrow0, bn, ybn);
        }
        mfma_v4f acc[RT][NB];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[rt][nb] = (mfma_v4f){0.f, 0.f, 0.f, 0.f};
        if constexpr (BF16) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    bf16x4 xb;
#pragma unroll
                    for (int j = 0; j < 4; ++j) xb[j] = to_bf16(b[rt][q][j]);
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[rt][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(qb[nb][q], xb, acc[rt][nb], 0, 0, 0);
                }
        } else {
#pragma unroll
            for (int s4 = 0; s4 < STEPS; ++s4)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const float bv = b[rt][s4 >> 2][s4 & 3];
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[rt][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[nb][s4], bv, acc[rt][nb], 0, 0, 0);
                }
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t t0 = row0 + 16 * rt;
            const int64_t row = t0 + n;
            const bool live = row < rows;
            if (projected) {
                // z^ of this lane's row: (y - X p) / rho, the dot in FP64 over
                // the lane's k values, then across the four lane groups
                double d = 0.0;
#pragma unroll
                for (int s4 = 0; s4 < STEPS; ++s4)
                    d += (double)b[rt][s4 >> 2][s4 & 3] * sp[16 * (s4 >> 2) + 4 * g + (s4 & 3)];
                d += __shfl_xor(d, 16);
                d += __shfl_xor(d, 32);
                const float yv = live ? yb[rt] : 0.0f;
                const float z = (float)(((double)yv - d) * inv_rho);
                if (live && g == 0) {
                    gfloat* A = (gfloat*)rq.A;
                    if (rq.kind == kRow) A[rq.m * rq.lda + row] = yv;
                    else A[row * rq.lda + rq.n] = yv;
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[rt][nb][r] += z * sqz[16 * nb + 4 * g + r];
            }
            if (live) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    if (16 * nb + 4 * g < ldo) *(gf4*)(Xo + t0 * ldo + 256 * nb + 64 * g + 4 * n) = acc[rt][nb];
            }
        }
        if constexpr (PF) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) b[rt][q] = bn[rt][q];
                yb[rt] = ybn[rt];
            }
        } else {
            if (t + 1 < TSTEPS) fetch(nrow0, b, yb);
        }
        row0 = nrow0;
    }
}

template <int KC, int ROWS, int RT, bool PF, bool BF16 = false>
__global__ void __launch_bounds__(kThreads) k_rotate_mfma_t(const Req* __restrict__ reqs,
                                                            const int* __restrict__ prefix, int nreq, int part) {
    // a grid sized for more tiles than this launch has (a captured tick,
    // sized for the streams' capacity) leaves the extra blocks idle
    if ((int)blockIdx.x >= prefix[nreq]) return;
    const int ri = find_req(prefix, nreq, blockIdx.x);
    rotate_mfma_t_block<KC, ROWS, RT, PF, BF16>(reqs + ri, blockIdx.x - prefix[ri], part);
}

// ---------------------------------------------------------------------------
// Deferred U (U = U0 W): materialisation and reset.
// k_defer_materialize: U[cur] <- U[cur] W[wpar][0:k, 0:k] in place (tiled,
// same ld; columns k.. zero): rows are independent and each block stages its
// 32 rows in LDS before writing them.  The buffer index stays, since V (rotated
// in place by deferred appends) lives in the same one.  W staged in LDS (FP64).
template <typename T, int KC>
__global__ void __launch_bounds__(256) k_defer_materialize(const DevHeader* __restrict__ hdr, T* U0, T* U1,
                                                           const double* W0, const double* W1, int64_t m) {
    __shared__ double sW[KC * KC];
    __shared__ double sX[32 * KC];
    const int k = hdr->k, ld = hdr->ld, cur = hdr->cur;
    const double* W = hdr->wpar ? W1 : W0;
    T* X = cur ? U1 : U0;
    T* Y = X;
    for (int e = threadIdx.x; e < k * k; e += 256) sW[(e / k) * KC + e % k] = W[(size_t)(e / k) * KC + e % k];
    const int64_t r0 = (int64_t)blockIdx.x * 32;
    const int nr = (int)min((int64_t)32, m - r0);
    for (int e = threadIdx.x; e < nr * k; e += 256) {
        const int rr = e / k, c = e - (e / k) * k;
        sX[rr * KC + c] = (double)X[uvo(r0 + rr, c, ld)];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * ld; e += 256) {
        const int rr = e / ld, j = e - (e / ld) * ld;
        double a = 0.0;
        if (j < k)
            for (int c = 0; c < k; ++c) a += sX[rr * KC + c] * sW[c * KC + j];
        Y[uvo(r0 + rr, j, ld)] = (T)a;
    }
}

// After a materialisation or a refresh: W and W^-1 of the current parity back
// to I (flip = 1 would also switch the current U / V buffers).
__device__ inline void defer_reset_body(DevHeader* hdr, double* W0, double* W1, double* Wi0, double* Wi1, int kc,
                                        int flip) {
    const int wp = hdr->wpar;
    double* W = wp ? W1 : W0;
    double* Wi = wp ? Wi1 : Wi0;
    for (int e = threadIdx.x; e < kc * kc; e += 256) {
        const double v = (e / kc == e - (e / kc) * kc) ? 1.0 : 0.0;
        W[e] = v;
        Wi[e] = v;
    }
    __syncthreads();
    if (flip && threadIdx.x == 0) hdr->cur ^= 1;
}
__global__ void __launch_bounds__(256) k_defer_reset(DevHeader* hdr, double* W0, double* W1, double* Wi0, double* Wi1,
                                                     int kc, int flip) {
    defer_reset_body(hdr, W0, W1, Wi0, Wi1, kc, flip);
}

}  // namespace isvd
