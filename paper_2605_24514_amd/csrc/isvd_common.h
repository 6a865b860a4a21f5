// Shared device/host definitions of the incremental-SVD engine (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isvd {

constexpr int kThreads = 256;      // threads of most blocks
constexpr int kProjTile = 256;     // basis rows per projection block
// basis rows per rotation block: the FP32 MFMA kernel walks 512 rows per
// block (4 waves x 16 rows x 8 steps) to amortise loading Q into registers;
// the FP64 LDS kernel takes 64 rows (16 for the widest bucket, so that Q and
// the row tile fit in LDS)
__host__ __device__ constexpr int rot_rows(int kc) { return kc <= 64 ? 64 : 16; }
constexpr int kMfmaRotRows = 512;
__host__ __device__ constexpr int rot_rows_for(int kc, bool fp64) { return fp64 ? rot_rows(kc) : kMfmaRotRows; }
constexpr int kMaxCore = 97;       // largest core order held in LDS (k <= 96)
constexpr int kMaxBlock = 96;      // largest refresh block size b

__host__ __device__ inline int round4(int k) { return (k + 3) & ~3; }

// Device-resident state of one stream (single source of truth for rank and
// buffer index, so that batched launches never need the host's view of k).
struct DevHeader {
    int32_t k;            // current rank
    int32_t ld;           // leading dimension of the current U / V buffers (= round4(k))
    int32_t cur;          // which of the two U / V buffers is current
    int32_t status;       // 0, or the error of the first rejected request; while
                          // set, every further update of the stream is rejected
    int64_t t;            // updates applied
    int64_t m, n;         // shape of A_t (authoritative; the host mirrors it)
    int64_t n_rejected;
    double N;             // ||A_t||_F^2
    double rho, xnorm, novelty, sigma_dropped;
    double sigma2;        // sum of the kept sigma^2
    double sigma_last;    // smallest kept sigma
    int32_t sweeps;       // Jacobi sweeps of the last core (-1: sweep cap reached)
    int32_t new_dir;      // last append had rho > tol
    int32_t last_kind;    // kind of the last applied update
    int32_t ref_k;        // rank of U_ref (stored at the last refresh that kept a reference)
    int32_t ref_ld;       // its leading dimension
    int32_t pad;
    int64_t ref_m;        // its rows
    double angle_ref;     // theta_ref (angle-threshold streams), radians
};

// Written by the core kernel of a request, read by its rotation kernel.
struct ReqScratch {
    int32_t skip;         // request rejected: the rotation writes nothing
    int32_t k_in, ld_in, k_out, ld_out, in_idx;
    double inv_rho;       // 1 / rho, or 0 when the residual is not a new direction
};

// One update request as the kernels see it.  Geometry is the pre-update
// shape (known exactly on the host); the rank comes from the DevHeader.
struct Req {
    int64_t m, n, lda;
    int64_t i, j;
    double delta, tol_rel;
    int32_t kind, k_keep;
    int32_t proj_tiles;   // blocks of each projection pass (0 for entry updates)
    int32_t rot_tiles_u;  // rotation blocks over U's rows (V's follow)
    DevHeader* hdr;
    ReqScratch* rs;
    void* A;
    void* U[2];
    void* V[2];
    double* S;            // singular values (k_cap + 1)
    double* p;            // pass-1 sums: p1[0..k), ||y||^2 at [kc], non-finite count at [kc+1]
    double* p2;           // pass-2 sums: p2[0..k), ||z1||^2 at [kc]
    double* partials;     // per-block partial sums, stride kc + 2
    unsigned* counters;   // arrival counters of the two projection passes
    void* QU;             // (k_in + 1) x ld_out rotation of U (row-major)
    void* QV;             // (k_in + 1) x ld_out rotation of V
    const void* payload;  // x (length n) or y (length m), storage type
};

enum { kRow = 0, kCol = 1, kEntry = 2 };

}  // namespace isvd
