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
// Block shapes of the FP32 matrix-core rotation (autotuned per rank bucket):
// rows per block, 16-row tiles per wave step, next-step prefetch.
struct RotVariant { int rows, rt, pf; };
constexpr int kRotVariants = 5;
constexpr RotVariant kRotVariant[kRotVariants] = {{256, 1, 1}, {512, 1, 1}, {1024, 1, 1}, {1024, 2, 0}, {2048, 2, 0}};
// V rotations of a tick (FP32, buckets up to 64) take 256 rows per block
// (four steps per wave): V has at most a few thousand rows, so the U shapes
// would leave a handful of blocks per stream, each walking its rows in turn
constexpr int kRotRowsV = 256;
constexpr int kMaxRank = 128;      // largest rank k of a stream
constexpr int kMaxCore = kMaxRank + 1;   // largest core order (an append's (k + 1) x (k + 1))
constexpr int kMaxBlock = 128;     // largest refresh block size b

__host__ __device__ inline int round4(int k) { return (k + 3) & ~3; }

// HBM layout of every basis (U, V, U_ref; leading dimension ld = a multiple
// of 4 >= k): 16-row tiles of 16 ld elements each; inside a tile, panels of
// 16 columns, and inside a panel the 4-column groups one after another, each
// holding its 16 rows x 4 columns row by row.  Element (r, c) lives at
//   (r / 16) 16 ld + (c / 16) 256 + ((c % 16) / 4) 64 + (r % 16) 4 + c % 4.
// Four consecutive columns c0..c0+3 (c0 % 4 == 0) of a row are contiguous
// (16 B in FP32), and one 4-column group of a 16-row tile is 64 contiguous
// elements: a wave reads it with one dwordx4 per lane (lane = group-local
// row + 16 x group), which is the matrix-core operand layout of the FP32
// rotation.  A tile is contiguous, so tiles are copied as blocks; buffers
// hold whole tiles (rows rounded up to 16).
__host__ __device__ inline int64_t uvo(int64_t r, int c, int ld) {
    return (r >> 4) * 16 * (int64_t)ld + (c >> 4) * 256 + ((c & 15) >> 2) * 64 + (r & 15) * 4 + (c & 3);
}
// Global-memory view of a pointer taken from a request or header record.
// Loads and stores through generic pointers are flat accesses, which count
// against the LDS wait counter as well: every wait for an LDS result would
// also wait for them.  Through these the compiler emits global accesses.
#define ISVD_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ inline ISVD_GLOBAL T* gmem(T* p) { return (ISVD_GLOBAL T*)p; }
// plain vector types for loads through such pointers
typedef float gvec_f4 __attribute__((ext_vector_type(4)));
typedef double gvec_d2 __attribute__((ext_vector_type(2)));
typedef double gvec_d4 __attribute__((ext_vector_type(4)));
// (row, column) inside a tile of element e of that tile
__host__ __device__ inline void uv_tile_rc(int e, int* r, int* c) {
    const int rem = e & 255;
    *r = (rem & 63) >> 2;
    *c = (e >> 8) * 16 + (rem >> 6) * 4 + (rem & 3);
}
__host__ __device__ inline int64_t round16(int64_t m) { return (m + 15) & ~(int64_t)15; }

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
    int32_t wpar;         // deferred U: which of the two W / W^-1 buffers is current
    int64_t ref_m;        // its rows
    double angle_ref;     // theta_ref (angle-threshold streams), radians
    // drift signals of the last applied update (no access to A needed):
    // largest principal angle between the previous and the new span of U
    // (the previous one zero-padded to the new rows), the same for V, and
    // ||sigma_t - sigma_{t-1}||_2 / ||sigma_{t-1}||_2 (zero-padded)
    double step_angle_u, step_angle_v, spec_change;
};

// Written by the core kernel of a request, read by its rotation kernel.
struct ReqScratch {
    int32_t skip;         // request rejected: the rotation writes nothing
    int32_t k_in, ld_in, k_out, ld_out, in_idx;
    int32_t deferred;     // row append applied to W (U = U0 W): no U rotation, V rotates in place
    double inv_rho;       // 1 / rho, or 0 when the residual is not a new direction
};

// One update request as the kernels see it.  Geometry is the pre-update
// shape (known exactly on the host); the rank comes from the DevHeader.
// The request (index in its list) and tile of one block of a merged launch.
struct BlockRef {
    int req, tile;
};

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
    double* p;            // projection coefficients p = p1 + p2 of an append (written by the core)
    double* partials;     // projection pass 1: per-block partial sums, stride kc + 2
    double* partials2;    // projection pass 2: the same
    void* QU;             // (k_in + 1) x ld_out rotation of U (row-major)
    void* QV;             // (k_in + 1) x ld_out rotation of V
    const void* payload;  // x (length n) or y (length m), storage type
    // deferred U (Brand's U = U0 W): W and W^-1 (two buffers each, KC x KC
    // FP64, row-major) when the stream keeps U that way, else null;
    // defer: the host asks for this row append to be applied to W
    double* Wd[2];
    double* Wdi[2];
    int32_t defer;
    int32_t pad;
    // FP64 cores of the widest bucket: the accumulated Jacobi rotations J
    // (CoreShape<128>::NMAX x LDW doubles, column-major) in global memory,
    // since K and J together exceed the LDS
    double* Jg;
};

enum { kRow = 0, kCol = 1, kEntry = 2 };

}  // namespace isvd
