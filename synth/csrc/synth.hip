// Device side of the synthetic input generator (inputs only; none of the
// update method).  Produces the same factor-model entries as synth/philox.py
// and synth/factor_model.py: the same Philox4x32-10 counters, the same
// 53-bit uniforms, Box-Muller with the same operation order, and the factor
// sum in the same order with no fused multiply-adds (built with
// -ffp-contract=off).  Only log / sin / cos may differ from the host's in the
// last bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
}

__device__ inline double u53(uint32_t hi, uint32_t lo) {
    double a = (double)(hi >> 5);
    double b = (double)(lo >> 6);
    return (a * 67108864.0 + b) * (1.0 / 9007199254740992.0);
}

// normals 2*block and 2*block+1 of (seed, stream, purpose, tick)
__device__ inline void normal_pair(uint32_t seed, uint32_t stream, uint32_t purpose, uint32_t tick,
                                   uint64_t block, double* z0, double* z1) {
    uint32_t c[4] = {(uint32_t)block, (uint32_t)(block >> 32), purpose, tick};
    philox10(c, seed, stream);
    double ua = u53(c[0], c[1]);
    double ub = u53(c[2], c[3]);
    double r = sqrt(-2.0 * log(1.0 - ua));
    double phi = 6.283185307179586 * ub;
    *z0 = r * cos(phi);
    *z1 = r * sin(phi);
}

__device__ inline double normal_at(uint32_t seed, uint32_t stream, uint32_t purpose, uint32_t tick, uint64_t idx) {
    double z0, z1;
    normal_pair(seed, stream, purpose, tick, idx >> 1, &z0, &z1);
    return (idx & 1) ? z1 : z0;
}

constexpr uint32_t P_LOAD = 1, P_FACT = 2, P_NOISE_ROW = 3;

// F[r][l] = sqrt(lam_l) * normal(FACT, tick = row0 + r)[l]
__global__ void k_factors(double* F, int64_t row0, int64_t rows, int K, const double* lam, uint32_t seed,
                          uint32_t stream) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * K) return;
    int64_t r = e / K;
    int l = (int)(e % K);
    F[e] = normal_at(seed, stream, P_FACT, (uint32_t)(row0 + r), (uint64_t)l) * sqrt(lam[l]);
}

// B[j][l] = normal(LOAD, tick = j)[l]
__global__ void k_loadings(double* B, int64_t cols, int K, uint32_t seed, uint32_t stream) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cols * K) return;
    int64_t j = e / K;
    int l = (int)(e % K);
    B[e] = normal_at(seed, stream, P_LOAD, (uint32_t)j, (uint64_t)l);
}

// out[r][j] = sum_l F[r][l] B[j][l] + noise * normal(NOISE_ROW, tick = row0 + r)[j]
// one thread per pair of columns (one Philox block)
template <typename T>
__global__ void k_rows(T* out, int64_t ld, const double* F, const double* B, int64_t rows, int64_t cols, int K,
                       double noise, int64_t row0, uint32_t seed, uint32_t stream) {
    const int64_t pairs = (cols + 1) / 2;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * pairs) return;
    int64_t r = e / pairs;
    int64_t blk = e % pairs;
    double z[2];
    normal_pair(seed, stream, P_NOISE_ROW, (uint32_t)(row0 + r), (uint64_t)blk, &z[0], &z[1]);
    for (int h = 0; h < 2; ++h) {
        int64_t j = 2 * blk + h;
        if (j >= cols) break;
        double acc = 0.0;
        for (int l = 0; l < K; ++l) acc = acc + F[r * K + l] * B[j * K + l];
        out[r * ld + j] = (T)(acc + noise * z[h]);
    }
}

}  // namespace

extern "C" {

// Rows [row0, row0 + rows) of stream (seed, stream)'s panel with `cols`
// columns (entries created by those rows): out is rows x cols, leading
// dimension ld, float (dtype 0) or double (dtype 1), device memory.
// F (rows x K), B (cols x K) and L (the K factor variances) are device
// buffers; the launches are queued on st.
static hipError_t synth_launch(void* out, int64_t ld, int32_t dtype, int64_t row0, int64_t rows, int64_t cols,
                               uint32_t seed, uint32_t stream, int32_t K, const double* L, double noise, double* F,
                               double* B, hipStream_t st) {
    k_factors<<<(unsigned)((rows * K + 255) / 256), 256, 0, st>>>(F, row0, rows, K, L, seed, stream);
    k_loadings<<<(unsigned)((cols * K + 255) / 256), 256, 0, st>>>(B, cols, K, seed, stream);
    const int64_t work = rows * ((cols + 1) / 2);
    if (dtype == 1)
        k_rows<double><<<(unsigned)((work + 255) / 256), 256, 0, st>>>((double*)out, ld, F, B, rows, cols, K, noise,
                                                                      row0, seed, stream);
    else
        k_rows<float><<<(unsigned)((work + 255) / 256), 256, 0, st>>>((float*)out, ld, F, B, rows, cols, K, noise,
                                                                     row0, seed, stream);
    return hipGetLastError();
}

// As above; lam: K factor variances (host).  Allocates its buffers and
// waits for the stream.  Returns 0 or a hipError_t value.
int synth_rows(void* out, int64_t ld, int32_t dtype, int64_t row0, int64_t rows, int64_t cols, uint32_t seed,
               uint32_t stream, int32_t K, const double* lam, double noise, void* hip_stream) {
    hipStream_t st = (hipStream_t)hip_stream;
    double *F = nullptr, *B = nullptr, *L = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&F, sizeof(double) * rows * K)) != hipSuccess) return (int)e;
    if ((e = hipMalloc(&B, sizeof(double) * cols * K)) != hipSuccess) { (void)hipFree(F); return (int)e; }
    if ((e = hipMalloc(&L, sizeof(double) * K)) != hipSuccess) { (void)hipFree(F); (void)hipFree(B); return (int)e; }
    e = hipMemcpyAsync(L, lam, sizeof(double) * K, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = synth_launch(out, ld, dtype, row0, rows, cols, seed, stream, K, L, noise, F, B, st);
    hipError_t e2 = hipStreamSynchronize(st);
    (void)hipFree(F);
    (void)hipFree(B);
    (void)hipFree(L);
    return (int)(e != hipSuccess ? e : e2);
}

// The same rows, queued on hip_stream without allocating or waiting: L_dev
// (the K factor variances), F_dev (at least rows x K) and B_dev (at least
// cols x K) are device buffers of the caller, reused only in stream order.
int synth_rows_async(void* out, int64_t ld, int32_t dtype, int64_t row0, int64_t rows, int64_t cols, uint32_t seed,
                     uint32_t stream, int32_t K, const double* L_dev, double noise, double* F_dev, double* B_dev,
                     void* hip_stream) {
    return (int)synth_launch(out, ld, dtype, row0, rows, cols, seed, stream, K, L_dev, noise, F_dev, B_dev,
                             (hipStream_t)hip_stream);
}

}  // extern "C"
