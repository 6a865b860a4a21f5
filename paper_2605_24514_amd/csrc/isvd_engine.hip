// libisvd: host side of the MI355X incremental-SVD engine and its C ABI.
//
// Per stream the engine keeps, in one device allocation:
//   A (m_cap x round4(n_cap), row-major), U and V in two buffers each (ping-pong:
//   every rotation writes the other buffer, so the leading dimension can
//   follow the rank), Sigma, the device header (rank, buffer index, N_t,
//   trackers), the rotation matrices of the last core, projection sums and
//   per-block partials, and a payload staging area.
// Updates are a fixed launch sequence (projection pass 1, pass 2, core,
// rotation) over request lists; a single update and a batched tick of many
// streams use the same kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>
#include <thread>
#include <vector>

#include "../../include/isvd.h"
#include "isvd_common.h"
#include "isvd_update.h"
#include "isvd_chain.h"
#include "isvd_segment.h"
#include "isvd_refresh.h"
#include "isvd_gcf.h"
#include "isvd_track.h"
#include "isvd_finance.h"

using namespace isvd;

// Workspace of isvd_refresh_noalloc: one static device array per GPU the
// library runs on, held until the process ends.  In host code its name is
// not a device address; its address on each device comes from
// hipGetSymbolAddress (noalloc_scratch_ptr).
constexpr size_t kNoAllocScratchBytes = (size_t)ISVD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_err;

isvd_status fail(isvd_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ISVD_E_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                               \
    } while (0)

#define ST_TRY(expr)                     \
    do {                                 \
        isvd_status s_ = (expr);         \
        if (s_ != ISVD_OK) return s_;    \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int bucket_for(int kmax) {
    if (kmax <= 8) return 8;
    if (kmax <= 16) return 16;
    if (kmax <= 32) return 32;
    if (kmax <= 64) return 64;
    return 128;
}

// ------------------------------------------------------------------ streams
struct Layout {
    size_t hdr, rs, S, p, partials, partials2, QU, QV, stage, U0, U1, V0, V1, Uref, TM, TH, TP, TS, Jg, A, total;
    size_t a_bytes = 0;      // A's bytes; with a_on_host, outside `total` (the device allocation)
    size_t rs_b, p_b, q_b;   // bytes of one copy of the double-buffered rs, p and QU / QV
};

constexpr int kMaxLiveStreams = 16384;   // capacity of an engine's header array

// A refresh workspace.  A lane's buffer that has to grow is retired, not
// freed (work queued on other lanes may still be running); retired buffers
// are freed where every lane is known to be idle.
struct WsBuf {
    char* p = nullptr;
    size_t bytes = 0;
    bool defer_free = false;
    bool fixed = false;    // caller-provided memory: never grown or freed
    std::vector<char*> retired;
};

struct Stream {
    isvd_config cfg;
    int esz = 4;          // bytes per storage element
    bool bf16 = false;    // rotations on the BF16 matrix cores
    int kc = 64;          // rank bucket (capacity of U / V rows)
    int k_target = 0;     // rank the truncation keeps
    int64_t m = 0, n = 0, t = 0;
    int64_t n_refresh = 0, t_last = 0;
    int64_t ntiles_max = 0;
    char* base = nullptr;
    size_t base_bytes = 0;      // size of the block holding base (a reused block may be larger)
    Layout L{};
    DevHeader* hdr = nullptr;   // the stream's entry of the engine's header array
    int slot = -1;              // its index there
    // per-update scratch read by the rotations, double-buffered by the parity
    // of the stream's update count: a U rotation may still run while the
    // stream's next core writes the other copy
    ReqScratch* rs[2] = {nullptr, nullptr};
    double* p[2] = {nullptr, nullptr};
    void* QU[2] = {nullptr, nullptr};
    void* QV[2] = {nullptr, nullptr};
    double *S = nullptr, *partials = nullptr, *partials2 = nullptr;
    void *stage = nullptr, *A = nullptr, *Uref = nullptr;
    double *TM = nullptr, *TH = nullptr, *TP = nullptr;   // angle trackers M, H and column-pass sums
    double* TS = nullptr;   // angle trackers: (kc + 1) x kc scratch of their updates
    double* Jg = nullptr;   // FP64 cores of bucket 128: their accumulated rotations
    void* U[2] = {nullptr, nullptr};
    void* V[2] = {nullptr, nullptr};
    hipEvent_t ev_u0 = nullptr, ev_u1 = nullptr, ev_r0 = nullptr, ev_r1 = nullptr;
    // a refresh fired by a tick runs on a refresh lane, after which ev_ready
    // fires; until then later work on the stream waits for it
    hipEvent_t ev_ready = nullptr;
    bool refreshing = false;
    // deferred U (U = U0 W): W, W^-1 (two parities each, kc x kc FP64) in one
    // allocation; defer_pending = row appends asked to go to W since U was
    // last explicit; defer_period = the appends between two explicit ones
    double* wbuf = nullptr;
    int64_t defer_pending = 0, defer_period = 1;
    bool have_update_time = false, have_refresh_time = false;
    bool live = false;
    bool grow_pending = false;   // adaptive rank: the next append keeps one more triplet
    bool angle = false;          // angle-threshold policy: trackers follow every update
    double last_ratio = 0.0;     // error policy: frob_ratio at its last check
    int refresh_rounds = 0;      // last refresh: Gram-form rounds (0: A form)
    bool refresh_converged = true;
    double drift_acc = 0.0;      // drift policy: step angles of U since the last refresh
    void* a_host = nullptr;      // A in pinned host memory (a_on_host)
};

// Leading dimension of A: n_cap rounded up to a multiple of 4, so that rows
// start 16-byte aligned (vector loads in the refresh products).
inline int64_t lda_of(const isvd_config& c) { return (c.n_cap + 3) & ~(int64_t)3; }

Layout make_layout(const isvd_config& c, int esz, int kc, int64_t* ntiles_max) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const int64_t mx = std::max(c.m_cap, c.n_cap);
    const int64_t nt = cdiv(mx, kProjTile);
    *ntiles_max = nt;
    L.rs_b = align_up(sizeof(ReqScratch), 256);
    L.rs = take(2 * L.rs_b);
    L.S = take(sizeof(double) * (kc + 2));
    L.p_b = align_up(sizeof(double) * (kc + 4), 256);
    L.p = take(2 * L.p_b);
    L.partials = take(sizeof(double) * (size_t)nt * (kc + 2));
    L.partials2 = take(sizeof(double) * (size_t)nt * (kc + 2));
    L.q_b = align_up((size_t)esz * (kc + 1) * kc, 256);
    L.QU = take(2 * L.q_b);
    L.QV = take(2 * L.q_b);
    L.stage = take((size_t)esz * mx);
    // bases hold whole 16-row tiles
    L.U0 = take((size_t)esz * round16(c.m_cap) * kc);
    L.U1 = take((size_t)esz * round16(c.m_cap) * kc);
    L.V0 = take((size_t)esz * round16(c.n_cap) * kc);
    L.V1 = take((size_t)esz * round16(c.n_cap) * kc);
    L.Uref = take((size_t)esz * round16(c.m_cap) * kc);
    const bool angle = c.policy.kind == ISVD_POL_ANGLE;
    L.TM = take(angle ? sizeof(double) * kc * kc : 0);
    L.TH = take(angle ? sizeof(double) * kc * kc : 0);
    L.TP = take(angle ? sizeof(double) * (size_t)cdiv(c.m_cap, kTrackRows) * (2 * kc + 1) : 0);
    L.TS = take(angle ? sizeof(double) * (size_t)(kc + 1) * kc : 0);   // tracker scratch
    L.Jg = take(esz == 8 ? sizeof(double) * core_jg_doubles(kc) : 0);
    L.A = take((size_t)esz * c.m_cap * lda_of(c));
    L.total = off;
    L.a_bytes = L.total - L.A;
    if (c.a_on_host) L.total = L.A;
    return L;
}

// ------------------------------------------------------- launch staging ring
// One upload buffer of the request ring: a fixed-stride piece of the ring's
// pinned host arena and of its device arena.
struct Slot {
    char* host = nullptr;
    char* dev = nullptr;
    hipEvent_t ev = nullptr;
    bool used = false;
};

// A group of requests of one (storage type, rank bucket), laid out in a slot.
struct Group {
    bool fp64;
    bool bf16 = false;         // FP32 storage, BF16 rotation products
    int kc;
    int rows = 0;              // rotation rows per block
    int rows_v() const { return (!fp64 && !bf16 && kc <= 64) ? kRotRowsV : rows; }   // ... of V-only launches
    int var = 1;               // FP32 rotation block shape (kRotVariant index)
    std::vector<Req> all;      // core + rotation list
    std::vector<Req> proj;     // row / column appends
    std::vector<int> pre_proj; // block prefix of the projection list (size proj+1)
    std::vector<int> pre_rot;  // block prefix of the rotation list, U and V (size all+1)
    std::vector<int> pre_rotU; // ... U tiles only
    std::vector<int> pre_rotV; // ... V tiles only
    std::vector<BlockRef> tproj, trotv;   // merged launches: request and tile of each block
    size_t off_tp = 0, off_tv = 0;
    size_t off_all = 0, off_proj = 0, off_pp = 0, off_pr = 0, off_pru = 0, off_prv = 0;
    bool proj_alias = false;   // the projection list is the whole list (no entry update)
    std::vector<isvd_id> ids;  // the requests' streams (the key of a captured tick)
    int rotU_cap = 0;          // U-rotation blocks at the streams' row capacity
    int grid_u = 0;            // > 0: U-rotation grid of a captured tick (extra blocks idle)
};

// A captured tick: the launch sequence of one set of row-append requests
// (streams, buckets, block shapes) recorded once as a HIP graph, replayed
// every tick with that tick's request records.  kTickGraphBufs buffers
// (pinned host and device) and as many graphs rotate, so that the host
// writes the records of later ticks while earlier ones still run.  Grids come from the streams'
// capacity (U rotation) or fixed shapes (projections, cores, V rotation).
constexpr int kTickGraphBufs = 8;   // ticks a host may run ahead of the device
struct TickGraph {
    std::vector<int64_t> key;
    size_t bytes = 0;
    char* host[kTickGraphBufs] = {};
    char* dev[kTickGraphBufs] = {};
    hipGraph_t graph[kTickGraphBufs] = {};
    hipGraphExec_t exec[kTickGraphBufs] = {};
    hipEvent_t done[kTickGraphBufs] = {};
    bool launched[kTickGraphBufs] = {};
    int next = 0;
    uint64_t last_use = 0;
};

}  // namespace

namespace {
struct LaunchRec {
    int32_t phase, kc, fp64, nreq;
    int64_t blocks;
    hipEvent_t b, e;
};
}  // namespace

struct isvd_engine {
    int device = 0;
    bool profiling = false;
    // Rotation lane (a stream of default priority): the U rotations of a
    // tick run there, each after its group's core, while the caller's
    // stream goes on with the next group and -- for ticks of row appends
    // only -- with the next tick's projections and cores.  The next core of
    // a stream needs V, Sigma and the header, never U, and writes the other
    // copy of the double-buffered scratch.  rot_pending: the lane has work
    // that no caller stream waits for yet; every call that reads or replaces
    // U first orders the caller's stream after it (join).
    hipStream_t rot_lane = nullptr;
    // second rotation lane: the U rotations of the buckets below 64, so that
    // they overlap the widest bucket's; the rotation lane joins it at the
    // end of every tick, so waiting for the rotation lane covers both
    hipStream_t rot_lane_b = nullptr;
    hipEvent_t ev_rot_b = nullptr;     // rotation lane b's part of a tick is done
    // second update lane: the rank buckets up to 32 run their projections,
    // cores and V rotations there, concurrently with the wider buckets on the
    // caller's stream (the assignment depends on the bucket only, so a
    // stream's updates stay on one lane)
    hipStream_t lane_b = nullptr;
    // first update lane (the wider buckets).  Both update lanes are the
    // engine's own streams, created one after the other so that they land on
    // different hardware queues whatever queue the caller's stream shares.
    hipStream_t lane_a = nullptr;
    // third update lane (deferred U: the 16- and 8-column buckets)
    hipStream_t lane_c = nullptr;
    hipEvent_t ev_c_end = nullptr;     // lane c's part of a tick is done
    hipEvent_t ev_fork = nullptr;      // the tick's request upload is done
    hipEvent_t ev_b_end = nullptr;     // lane b's part of a tick is done
    std::vector<hipEvent_t> ev_core;   // per group of a tick: its core is done
    hipEvent_t ev_main = nullptr;      // lane a's part of a tick is done
    hipEvent_t ev_rot = nullptr;       // join point of the rotation lane
    hipEvent_t ev_tick_end[2] = {nullptr, nullptr};   // by tick parity
    uint64_t ticks = 0;
    int lane_ticks = 0;                // consecutive ticks run without the rotation lanes
    std::vector<uint64_t> seen_stamp;  // per stream id: the tick call that last named it
    uint64_t stamp = 0;
    bool rot_pending = false;
    bool pipelining = true;            // isvd_set_pipelining
    bool defer_u = false;              // isvd_set_deferred_u
    std::vector<LaunchRec> prof;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    uint64_t budget = 0, used = 0;
    std::vector<Stream*> streams;
    std::vector<Slot> ring;
    size_t ring_next = 0;
    char* ring_host = nullptr;         // pinned, ring.size() x ring_stride
    char* ring_dev = nullptr;          // device, ring.size() x ring_stride
    size_t ring_stride = 0;
    // refresh workspace (sized for the largest refresh so far)
    WsBuf ws;
    // exact-metrics workspace
    char* mws = nullptr;
    size_t mws_bytes = 0;
    // refresh lanes: the refreshes that the policies of one tick fire run
    // concurrently, each lane with its own stream (default priority) and
    // workspace
    struct RefreshLane {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;     // recorded after the lane's latest work
        bool pending = false;        // work queued since the last join
        WsBuf ws;
        WsBuf jobs;                  // job tables of the segmented batches on this lane
    };
    std::vector<RefreshLane> rlanes;
    int next_lane = 0;               // lane of the next stream-creation SVD
    hipEvent_t ev_policies = nullptr;
    int* dsweeps = nullptr;          // device: Rayleigh-Ritz sweep count per header slot
    int* rsweeps = nullptr;          // pinned copy
    // segmented refresh batches (isvd_set_segmented_refresh): the A-form
    // refreshes of FP32 streams that one tick fires, one launch per phase
    bool seg_refresh = true;
    int seg_lane = 0;                // refresh lane of the next batch (batches rotate over the lanes)
    struct SegSlot {
        char* host = nullptr;        // pinned staging of the job tables
        size_t bytes = 0;
        hipEvent_t ev = nullptr;     // after the copy out of it
        bool used = false;
    };
    SegSlot seg_slot[4];
    int seg_next = 0;
    WsBuf seg_cws, seg_cjobs;        // the batched error checks' workspaces and job tables
    double* chk_host = nullptr;      // pinned: their E_inc, ||A||^2 and Ritz values
    size_t chk_host_n = 0;
    // block cache (isvd_set_block_cache): device blocks of released streams,
    // by size, reused by later streams; each release records an event on
    // every engine stream, and a reusing stream creation waits for them
    size_t bcache_cap = 0, bcache_bytes = 0;
    std::multimap<size_t, char*> bcache;
    std::vector<hipEvent_t> ev_rel;
    std::vector<Stream*> releasing;  // released while their refresh still ran: cached once it ends
    std::vector<char*> to_free;      // blocks past the cap, freed together after one device wait
    // the device headers of all live streams, one array (a slot per stream),
    // so that a tick reads them back with one copy into the pinned mirror
    DevHeader* hdr_dev = nullptr;
    DevHeader* hdr_mirror = nullptr;
    int* chain_plan = nullptr;       // device plan of a merged tick's U rotations
    int hdr_hi = 0;                  // slots [0, hdr_hi) have been handed out
    std::vector<int> hdr_free;
    // block shape (kRotVariant index) of the FP32 matrix-core rotation per
    // rank bucket (8, 16, 32, 64; the widest bucket uses the LDS-staged
    // kernel), chosen by isvd_autotune
    int rot_var_f32[4] = {1, 1, 1, 1};
    // captured ticks (isvd_set_tick_graphs): cache of a few request sets
    bool tick_graphs = false;
    hipStream_t capture_st = nullptr;
    std::vector<TickGraph*> tgraphs;
};

namespace {

isvd_status ensure_device(isvd_engine* e) {
    HIP_TRY(hipSetDevice(e->device));
    return ISVD_OK;
}

// Device address of `scratch` on each device, looked up once per device
// with that device current (engine creation).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

isvd_status noalloc_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(ISVD_E_INVAL, "device %d", device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return ISVD_OK;
    void* ptr = nullptr;
    const hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (err != hipSuccess || !ptr)
        return fail(ISVD_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(err));
    g_scratch_ptr[device] = (char*)ptr;
    return ISVD_OK;
}

isvd_status get_stream(isvd_engine* e, isvd_id id, Stream** out) {
    if (!e) return fail(ISVD_E_INVAL, "null engine");
    if (id < 0 || id >= (isvd_id)e->streams.size() || !e->streams[id] || !e->streams[id]->live)
        return fail(ISVD_E_STATE, "unknown or released stream id %lld", (long long)id);
    *out = e->streams[id];
    return ISVD_OK;
}

template <typename K>
isvd_status allow_lds(K kern, size_t bytes) {
    HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return ISVD_OK;
}


size_t sym_norm2_lds(int k) { return sizeof(double) * (size_t)((k + 1) * WideShape::LDW + k); }

// Acquire a staging slot of at least `bytes`; waits for its previous use.
// Upload of a slot: the GPU reads the pinned host arena directly.  A kernel
// on the stream orders itself after that stream's waits on the device,
// where an asynchronous copy behind a cross-stream wait was seen to hold
// the calling thread until the wait resolved.
__global__ void __launch_bounds__(256) k_upload(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n16) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

// bytes: a multiple of 16 (every slot layout ends on a 64-byte boundary)
isvd_status upload_slot(const Slot* slot, size_t bytes, hipStream_t st) {
    const size_t n16 = align_up(bytes, 16) / 16;
    if (n16 == 0) return ISVD_OK;
    const int blocks = (int)std::min<size_t>(cdiv(n16, 256), 64);
    k_upload<<<blocks, 256, 0, st>>>(reinterpret_cast<const uint4*>(slot->host), reinterpret_cast<uint4*>(slot->dev),
                                      n16);
    HIP_TRY(hipGetLastError());
    return ISVD_OK;
}

isvd_status acquire_slot(isvd_engine* e, size_t bytes, Slot** out) {
    if (bytes > e->ring_stride) {
        // every slot grows at once (geometrically, so a handful of times per
        // engine): the slots still in flight drain first, then both arenas
        // are replaced; a tick never allocates otherwise
        for (Slot& s : e->ring)
            if (s.used) {
                HIP_TRY(hipEventSynchronize(s.ev));
                s.used = false;
            }
        const size_t stride = align_up(std::max({2 * bytes, 2 * e->ring_stride, (size_t)65536}), 4096);
        if (e->ring_host) HIP_TRY(hipHostFree(e->ring_host));
        if (e->ring_dev) HIP_TRY(hipFree(e->ring_dev));
        e->ring_host = e->ring_dev = nullptr;
        e->ring_stride = 0;
        for (Slot& s : e->ring) s.host = s.dev = nullptr;
        HIP_TRY(hipHostMalloc((void**)&e->ring_host, stride * e->ring.size(), hipHostMallocDefault));
        HIP_TRY(hipMalloc((void**)&e->ring_dev, stride * e->ring.size()));
        e->ring_stride = stride;
        for (size_t i = 0; i < e->ring.size(); ++i) {
            e->ring[i].host = e->ring_host + i * stride;
            e->ring[i].dev = e->ring_dev + i * stride;
        }
    }
    Slot& s = e->ring[e->ring_next];
    e->ring_next = (e->ring_next + 1) % e->ring.size();
    if (s.used) HIP_TRY(hipEventSynchronize(s.ev));
    *out = &s;
    return ISVD_OK;
}

// ---------------------------------------------------------- kernel dispatch
template <typename T, int KC>
isvd_status launch_group_phase(const Group& g, const char* dev, int phase, hipStream_t st) {
    const Req* all = reinterpret_cast<const Req*>(dev + g.off_all);
    const Req* proj = reinterpret_cast<const Req*>(dev + g.off_proj);
    const int* pp = reinterpret_cast<const int*>(dev + g.off_pp);
    const int np = (int)g.proj.size(), na = (int)g.all.size();
    if (phase == 0 && np > 0) {
        k_proj<T, KC, 1><<<g.pre_proj[np], kThreads, 0, st>>>(proj, pp, np);
    } else if (phase == 1 && np > 0) {
        k_proj<T, KC, 2><<<g.pre_proj[np], kThreads, 0, st>>>(proj, pp, np);
    } else if (phase == 2 && na > 0) {
        size_t lds = sizeof(double) * core_lds_doubles<KC, sizeof(T) == 8>();
        k_core<T, KC><<<na, core_nt<KC, sizeof(T) == 8>(), lds, st>>>(all);
    } else if (phase >= 3 && na > 0) {
        // 3: U tiles, 4: V tiles, 5: both
        const int part = phase == 3 ? 1 : phase == 4 ? 2 : 0;
        const int* pr = reinterpret_cast<const int*>(dev + (part == 1 ? g.off_pru : part == 2 ? g.off_prv : g.off_pr));
        const int nb = (part == 1 && g.grid_u > 0) ? g.grid_u
                                                    : (part == 1 ? g.pre_rotU : part == 2 ? g.pre_rotV : g.pre_rot)[na];
        if (nb == 0) return ISVD_OK;
        if constexpr (sizeof(T) == 4 && KC <= 64) {
            static_assert(kRotVariants == 5, "variant dispatch");
            if (g.bf16) {
                k_rotate_mfma_t<KC, 512, 1, true, true><<<nb, kThreads, 0, st>>>(all, pr, na, part);
                HIP_TRY(hipGetLastError());
                return ISVD_OK;
            }
            if (part == 2) {
                k_rotate_mfma_t<KC, kRotRowsV, 1, true><<<nb, kThreads, 0, st>>>(all, pr, na, part);
                HIP_TRY(hipGetLastError());
                return ISVD_OK;
            }
            switch (g.var) {
                case 0: k_rotate_mfma_t<KC, 256, 1, true><<<nb, kThreads, 0, st>>>(all, pr, na, part); break;
                case 2: k_rotate_mfma_t<KC, 1024, 1, true><<<nb, kThreads, 0, st>>>(all, pr, na, part); break;
                case 3: k_rotate_mfma_t<KC, 1024, 2, false><<<nb, kThreads, 0, st>>>(all, pr, na, part); break;
                case 4: k_rotate_mfma_t<KC, 2048, 2, false><<<nb, kThreads, 0, st>>>(all, pr, na, part); break;
                default: k_rotate_mfma_t<KC, 512, 1, true><<<nb, kThreads, 0, st>>>(all, pr, na, part); break;
            }
        } else if constexpr (sizeof(T) == 4) {
            if (g.bf16)   // BF16 products, transposed form (Q^T in registers as BF16)
                k_rotate_mfma_t<KC, kMfmaRotRows, 1, true, true><<<nb, kThreads, 0, st>>>(all, pr, na, part);
            else
                k_rotate_mfma<KC><<<nb, kThreads, 0, st>>>(all, pr, na, part);
        } else {
            k_rotate<T, KC><<<nb, kThreads, 0, st>>>(all, pr, na, part);
        }
    }
    HIP_TRY(hipGetLastError());
    return ISVD_OK;
}

isvd_status launch_phase(const Group& g, const char* dev, int phase, hipStream_t st) {
    if (g.fp64) {
        switch (g.kc) {
            case 8: return launch_group_phase<double, 8>(g, dev, phase, st);
            case 16: return launch_group_phase<double, 16>(g, dev, phase, st);
            case 32: return launch_group_phase<double, 32>(g, dev, phase, st);
            case 64: return launch_group_phase<double, 64>(g, dev, phase, st);
            default: return launch_group_phase<double, 128>(g, dev, phase, st);
        }
    }
    switch (g.kc) {
        case 8: return launch_group_phase<float, 8>(g, dev, phase, st);
        case 16: return launch_group_phase<float, 16>(g, dev, phase, st);
        case 32: return launch_group_phase<float, 32>(g, dev, phase, st);
        case 64: return launch_group_phase<float, 64>(g, dev, phase, st);
        default: return launch_group_phase<float, 128>(g, dev, phase, st);
    }
}

template <typename T, int KC>
isvd_status set_lds_limits_for() {
    ST_TRY(allow_lds(k_core<T, KC>, sizeof(double) * core_lds_doubles<KC, sizeof(T) == 8>()));
    return ISVD_OK;
}

isvd_status set_lds_limits() {
    ST_TRY((set_lds_limits_for<float, 8>()));
    ST_TRY((set_lds_limits_for<float, 16>()));
    ST_TRY((set_lds_limits_for<float, 32>()));
    ST_TRY((set_lds_limits_for<float, 64>()));
    ST_TRY((set_lds_limits_for<float, 128>()));
    ST_TRY((set_lds_limits_for<double, 8>()));
    ST_TRY((set_lds_limits_for<double, 16>()));
    ST_TRY((set_lds_limits_for<double, 32>()));
    ST_TRY((set_lds_limits_for<double, 64>()));
    ST_TRY((set_lds_limits_for<double, 128>()));
    ST_TRY(allow_lds(k_core_chain, sizeof(double) * chain_core_lds()));
    ST_TRY(allow_lds(k_svd_small_noj<float>, sizeof(double) * svd_noj_lds_doubles()));
    ST_TRY(allow_lds(k_svd_small_noj<double>, sizeof(double) * svd_noj_lds_doubles()));
    ST_TRY(allow_lds(k_seg_svd, sizeof(double) * svd_noj_lds_doubles()));
    ST_TRY(allow_lds(k_sym_norm2, sym_norm2_lds(kMaxBlock)));
    ST_TRY(allow_lds(k_track<float>, sizeof(double) * track_lds_doubles()));
    ST_TRY(allow_lds(k_track<double>, sizeof(double) * track_lds_doubles()));
    ST_TRY(allow_lds(k_theta_tracks, sizeof(double) * theta_lds_doubles()));
    ST_TRY(allow_lds(k_theta_direct, sizeof(double) * theta_lds_doubles()));
    return ISVD_OK;
}

// Build the request a single stream's update sends to the kernels.
int bucket_index(int kc) { return kc <= 8 ? 0 : kc <= 16 ? 1 : kc <= 32 ? 2 : kc <= 64 ? 3 : 4; }

// rows per rotation block of a bucket
int var_for(const isvd_engine* e, int kc, bool fp64) { return (fp64 || kc > 64) ? 1 : e->rot_var_f32[bucket_index(kc)]; }

int rows_for(const isvd_engine* e, int kc, bool fp64) {
    if (fp64) return rot_rows(kc);
    if (kc > 64) return kMfmaRotRows;
    return kRotVariant[var_for(e, kc, fp64)].rows;
}

Req make_req(const isvd_engine* e, Stream& s, int kind, const void* payload, int64_t i, int64_t j, double delta,
             int k_keep) {
    Req r{};
    r.m = s.m;
    r.n = s.n;
    r.lda = lda_of(s.cfg);
    r.i = i;
    r.j = j;
    r.delta = delta;
    r.tol_rel = s.cfg.tol_rel;
    r.kind = kind;
    r.k_keep = k_keep;
    // appends: projection passes over row tiles of V (row) or U (column)
    r.proj_tiles = kind == kCol ? (int)cdiv(s.m, kProjTile) : kind == kRow ? (int)cdiv(s.n, kProjTile) : 0;
    r.rot_tiles_u = (int)cdiv(s.m, rows_for(e, s.kc, s.esz == 8));
    const int par = (int)(s.t & 1);
    r.hdr = s.hdr;
    r.rs = s.rs[par];
    r.A = s.A;
    r.U[0] = s.U[0];
    r.U[1] = s.U[1];
    r.V[0] = s.V[0];
    r.V[1] = s.V[1];
    r.S = s.S;
    r.p = s.p[par];
    r.partials = s.partials;
    r.partials2 = s.partials2;
    r.QU = s.QU[par];
    r.QV = s.QV[par];
    r.Jg = s.Jg;
    r.payload = payload;
    if (s.wbuf && e->defer_u) {
        const size_t w = (size_t)s.kc * s.kc;
        r.Wd[0] = s.wbuf;
        r.Wd[1] = s.wbuf + w;
        r.Wdi[0] = s.wbuf + 2 * w;
        r.Wdi[1] = s.wbuf + 3 * w;
        // row appends go to W between explicit ones, every defer_period-th
        // append rotates U (staggered over streams by their slot)
        if (kind == kRow) {
            r.defer = s.defer_pending + 1 < s.defer_period ? 1 : 0;
            s.defer_pending = r.defer ? s.defer_pending + 1 : 0;
        }
    }
    return r;
}

int rot_tiles(const Req& r, int rows) { return r.rot_tiles_u + (int)cdiv(r.n, rows); }

// ------------------------------------------------------------- deferred U
// FP32 storage, rank buckets up to 64, no tracker and no rank-changing or
// U-reading policy: row appends may go to W (U = U0 W) between explicit ones.
bool defer_eligible(const Stream& s) {
    const int pk = s.cfg.policy.kind;
    return s.esz == 4 && !s.bf16 && s.kc <= 64 && !s.angle && (pk == ISVD_POL_NONE || pk == ISVD_POL_PERIODIC);
}

__global__ void __launch_bounds__(256) k_eye4(double* buf, int kc) {
    const int w = kc * kc;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < 4 * w; e += gridDim.x * 256) {
        const int q = e % w;
        buf[e] = (q / kc == q % kc) ? 1.0 : 0.0;
    }
}

// explicit rotations every defer_period-th row append: the appends in between
// add about k / m each to the squared weight of W's smallest direction, so
// m / (8 k) of them keep W within a few percent of orthogonal
int64_t defer_period_for(const Stream& s) {
    return std::max<int64_t>(1, std::min<int64_t>(256, s.m / (8 * (int64_t)s.kc)));
}

isvd_status ensure_wbuf(Stream& s, hipStream_t st) {
    if (s.wbuf || !defer_eligible(s)) return ISVD_OK;
    const size_t bytes = sizeof(double) * 4 * (size_t)s.kc * s.kc;
    HIP_TRY(hipMalloc((void**)&s.wbuf, bytes));
    k_eye4<<<(int)std::min<int64_t>(64, cdiv(4 * s.kc * s.kc, 256)), 256, 0, st>>>(s.wbuf, s.kc);
    HIP_TRY(hipGetLastError());
    s.defer_period = defer_period_for(s);
    s.defer_pending = s.slot >= 0 ? (7 * (int64_t)s.slot) % s.defer_period : 0;
    return ISVD_OK;
}

template <int KC>
void launch_materialize(Stream& s, hipStream_t st) {
    const size_t w = (size_t)KC * KC;
    k_defer_materialize<float, KC><<<(int)cdiv(s.m, 32), 256, 0, st>>>(s.hdr, (float*)s.U[0], (float*)s.U[1], s.wbuf,
                                                                       s.wbuf + w, s.m);
}

// Make U explicit (U0 W in place, W = I) before anything that
// reads U: column appends, entry updates, factors, exact metrics.
isvd_status defer_flush(Stream& s, hipStream_t st) {
    if (!s.wbuf || s.defer_pending == 0) return ISVD_OK;
    switch (s.kc) {
        case 8: launch_materialize<8>(s, st); break;
        case 16: launch_materialize<16>(s, st); break;
        case 32: launch_materialize<32>(s, st); break;
        default: launch_materialize<64>(s, st); break;
    }
    const size_t w = (size_t)s.kc * s.kc;
    k_defer_reset<<<1, 256, 0, st>>>(s.hdr, s.wbuf, s.wbuf + w, s.wbuf + 2 * w, s.wbuf + 3 * w, s.kc, 0);
    HIP_TRY(hipGetLastError());
    s.defer_pending = 0;
    s.defer_period = defer_period_for(s);
    return ISVD_OK;
}

// A refresh writes U explicitly: W back to I.
isvd_status defer_after_refresh(Stream& s, hipStream_t st) {
    if (!s.wbuf) return ISVD_OK;
    const size_t w = (size_t)s.kc * s.kc;
    k_defer_reset<<<1, 256, 0, st>>>(s.hdr, s.wbuf, s.wbuf + w, s.wbuf + 2 * w, s.wbuf + 3 * w, s.kc, 0);
    HIP_TRY(hipGetLastError());
    s.defer_pending = 0;
    s.defer_period = defer_period_for(s);
    return ISVD_OK;
}

isvd_status next_event(isvd_engine* e, hipEvent_t* out) {
    if (e->ev_used == e->ev_pool.size()) {
        hipEvent_t ev;
        HIP_TRY(hipEventCreate(&ev));
        e->ev_pool.push_back(ev);
    }
    *out = e->ev_pool[e->ev_used++];
    return ISVD_OK;
}

isvd_status ensure_lanes(isvd_engine* e) {
    if (e->rot_lane) return ISVD_OK;
    HIP_TRY(hipStreamCreateWithFlags(&e->lane_a, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&e->lane_b, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&e->lane_c, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&e->rot_lane, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&e->ev_c_end, hipEventDisableTiming));
    HIP_TRY(hipStreamCreateWithFlags(&e->rot_lane_b, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&e->ev_rot_b, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&e->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&e->ev_b_end, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&e->ev_main, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&e->ev_rot, hipEventDisableTiming));
    for (int q = 0; q < 2; ++q) HIP_TRY(hipEventCreateWithFlags(&e->ev_tick_end[q], hipEventDisableTiming));
    return ISVD_OK;
}

// Order `st` after everything queued on the rotation lane.
isvd_status join(isvd_engine* e, hipStream_t st) {
    if (!e->rot_pending) return ISVD_OK;
    HIP_TRY(hipEventRecord(e->ev_rot, e->rot_lane));
    HIP_TRY(hipStreamWaitEvent(st, e->ev_rot, 0));
    e->rot_pending = false;
    return ISVD_OK;
}

isvd_status launch_recorded(isvd_engine* e, const Group& g, const char* dev, int phase, hipStream_t gs) {
    LaunchRec rec{};
    if (e->profiling) {
        ST_TRY(next_event(e, &rec.b));
        ST_TRY(next_event(e, &rec.e));
        HIP_TRY(hipEventRecord(rec.b, gs));
    }
    ST_TRY(launch_phase(g, dev, phase, gs));
    if (e->profiling) {
        HIP_TRY(hipEventRecord(rec.e, gs));
        const int np = (int)g.proj.size(), na = (int)g.all.size();
        rec.phase = phase;
        rec.kc = g.kc;
        rec.fp64 = g.fp64 ? 1 : 0;
        rec.nreq = phase < 2 ? np : na;
        rec.blocks = phase < 2 ? g.pre_proj[np] : phase == 2 ? na : phase == 3 ? g.pre_rotU[na] : g.pre_rotV[na];
        e->prof.push_back(rec);
    }
    return ISVD_OK;
}

// Lay out groups in a slot, upload, and launch one tick (or one immediate
// update).  The caller's stream uploads the requests and forks the update
// lanes.  Per group, on its update lane (lane a for buckets of 64 and
// wider; lane b for the others, or with deferred U lane b for bucket 32 and
// lane c for the narrower ones): the two projection passes, the
// core, then V's rotation; after the group's core, U's rotation on a
// rotation lane (rotation lane b for the buckets below 64, the rotation lane
// for the others, so the two overlap).
// pipelined: the caller's stream is not made to wait for the U rotations (a
// later join does); otherwise it is joined at the end.  Lane b is always
// joined into the caller's stream at the end of the tick: its launches read
// the payloads, and no U rotation of a pipelined tick does.  The rotation lane
// never runs more than one tick behind: a tick's first launch waits for the
// lane's end of the tick before last, whose scratch copy this tick's cores
// overwrite.
// Layout of a tick's groups in one upload buffer: block prefixes and offsets
// (groups sorted by bucket, widest first).  Returns the buffer's bytes.
size_t layout_groups(std::vector<Group>& groups, bool tables = false) {
    std::sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) {
        return a.kc != b.kc ? a.kc > b.kc : (a.fp64 && !b.fp64);
    });
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off = align_up(off + b, 64);
        return o;
    };
    for (Group& g : groups) {
        g.pre_proj.assign(g.proj.size() + 1, 0);
        for (size_t q = 0; q < g.proj.size(); ++q) g.pre_proj[q + 1] = g.pre_proj[q] + g.proj[q].proj_tiles;
        const size_t na = g.all.size();
        g.pre_rot.assign(na + 1, 0);
        g.pre_rotU.assign(na + 1, 0);
        g.pre_rotV.assign(na + 1, 0);
        for (size_t q = 0; q < na; ++q) {
            const int tu = g.all[q].rot_tiles_u, tv = (int)cdiv(g.all[q].n, g.rows);
            g.pre_rot[q + 1] = g.pre_rot[q] + tu + tv;
            g.pre_rotU[q + 1] = g.pre_rotU[q] + tu;
            g.pre_rotV[q + 1] = g.pre_rotV[q] + (int)cdiv(g.all[q].n, g.rows_v());
        }
        g.off_all = take(sizeof(Req) * na);
        // the projection list equals the whole list when every request is an
        // append (no entry update): then it is the same upload
        g.proj_alias = g.proj.size() == na;
        g.off_proj = g.proj_alias ? g.off_all : take(sizeof(Req) * g.proj.size());
        g.off_pp = take(sizeof(int) * g.pre_proj.size());
        g.off_pr = take(sizeof(int) * (na + 1));
        g.off_pru = take(sizeof(int) * (na + 1));
        g.off_prv = take(sizeof(int) * (na + 1));
        g.tproj.clear();
        g.trotv.clear();
        if (tables) {
            for (size_t q = 0; q < g.proj.size(); ++q)
                for (int t = 0; t < g.proj[q].proj_tiles; ++t) g.tproj.push_back({(int)q, t});
            for (size_t q = 0; q < na; ++q)
                for (int t = 0; t < g.pre_rotV[q + 1] - g.pre_rotV[q]; ++t) g.trotv.push_back({(int)q, t});
            g.off_tp = take(sizeof(BlockRef) * g.tproj.size());
            g.off_tv = take(sizeof(BlockRef) * g.trotv.size());
        }
    }
    return off;
}

// The groups' request records and prefixes into an upload buffer.
void fill_groups(const std::vector<Group>& groups, char* host) {
    for (const Group& g : groups) {
        const size_t na = g.all.size();
        if (na) memcpy(host + g.off_all, g.all.data(), sizeof(Req) * na);
        if (!g.proj.empty() && !g.proj_alias) memcpy(host + g.off_proj, g.proj.data(), sizeof(Req) * g.proj.size());
        memcpy(host + g.off_pp, g.pre_proj.data(), sizeof(int) * g.pre_proj.size());
        memcpy(host + g.off_pr, g.pre_rot.data(), sizeof(int) * (na + 1));
        memcpy(host + g.off_pru, g.pre_rotU.data(), sizeof(int) * (na + 1));
        memcpy(host + g.off_prv, g.pre_rotV.data(), sizeof(int) * (na + 1));
        if (!g.tproj.empty()) memcpy(host + g.off_tp, g.tproj.data(), sizeof(BlockRef) * g.tproj.size());
        if (!g.trotv.empty()) memcpy(host + g.off_tv, g.trotv.data(), sizeof(BlockRef) * g.trotv.size());
    }
}

// Deferred U (own lanes): the launch sequence of one tick whose records are
// uploaded from `host` to `dev` by the first launch on `st`: the update
// lanes fork from `st`, each group runs its projections, core, V and U
// rotations on its lane, and the lanes join back into `st`.
isvd_status own_lane_sequence(isvd_engine* e, const std::vector<Group>& groups, const char* host, char* dev,
                              size_t bytes, hipStream_t st) {
    const size_t n16 = align_up(bytes, 16) / 16;
    if (n16 > 0)
        k_upload<<<(int)std::min<size_t>(cdiv(n16, 256), 64), 256, 0, st>>>(reinterpret_cast<const uint4*>(host),
                                                                          reinterpret_cast<uint4*>(dev), n16);
    HIP_TRY(hipGetLastError());
    auto lane_of = [&](const Group& g) -> int { return g.kc >= 64 ? 0 : g.kc >= 32 ? 1 : 2; };
    constexpr int kLanes = 3;
    hipStream_t lanes[kLanes] = {e->lane_a, e->lane_b, e->lane_c};
    hipEvent_t lane_end[kLanes] = {e->ev_main, e->ev_b_end, e->ev_c_end};
    bool used[kLanes] = {false, false, false};
    for (const Group& g : groups) used[lane_of(g)] = true;
    HIP_TRY(hipEventRecord(e->ev_fork, st));
    for (int l = 0; l < kLanes; ++l)
        if (used[l]) HIP_TRY(hipStreamWaitEvent(lanes[l], e->ev_fork, 0));
    for (const Group& g : groups) {
        hipStream_t ln = lanes[lane_of(g)];
        for (int phase = 0; phase < 3; ++phase) ST_TRY(launch_recorded(e, g, dev, phase, ln));
        ST_TRY(launch_recorded(e, g, dev, 4, ln));
        ST_TRY(launch_recorded(e, g, dev, 3, ln));
    }
    for (int l = 0; l < kLanes; ++l)
        if (used[l]) {
            HIP_TRY(hipEventRecord(lane_end[l], lanes[l]));
            HIP_TRY(hipStreamWaitEvent(st, lane_end[l], 0));
        }
    return ISVD_OK;
}

// ------------------------------------------------ merged (chain) ticks
// A tick takes the merged launches (isvd_chain.h) when U is deferred and
// every group is an FP32 bucket of ranks up to 64: the tick is then one
// chain of kernels on the caller's stream, with no lanes to fork and join.
bool chain_ok(const isvd_engine* e, const std::vector<Group>& groups) {
    if (!e->defer_u || groups.empty() || groups.size() > (size_t)kChainMax) return false;
    size_t nreq = 0;
    for (const Group& g : groups) {
        if (g.fp64 || g.bf16 || g.kc > 64) return false;
        nreq += g.all.size();
    }
    return nreq <= (size_t)kChainMaxReqs;
}

isvd_status ensure_chain_plan(isvd_engine* e) {
    if (!e->chain_plan)
        HIP_TRY(hipMalloc((void**)&e->chain_plan, sizeof(int) * chain_plan_ints(kMaxLiveStreams)));
    return ISVD_OK;
}

// The request lists of one phase (0, 1: projection passes, 2: cores, 3: U,
// 4: V) of the groups laid out in `dev`, in the groups' order (widest bucket
// first); *blocks: the blocks of the merged launch.
MultiGroup chain_args(const std::vector<Group>& groups, const char* dev, int phase, int* blocks) {
    MultiGroup mg{};
    mg.begin[0] = 0;
    for (const Group& g : groups) {
        const int np = (int)g.proj.size(), na = (int)g.all.size();
        const int nreq = phase < 2 ? np : na;
        const int nb = phase < 2 ? g.pre_proj[np] : phase == 2 ? na : phase == 4 ? g.pre_rotV[na] : 0;
        if (nreq == 0 || (phase != 3 && nb == 0)) continue;
        const int q = mg.n++;
        mg.kc[q] = g.kc;
        mg.reqs[q] = reinterpret_cast<const Req*>(dev + (phase < 2 ? g.off_proj : g.off_all));
        mg.tbl[q] = reinterpret_cast<const BlockRef*>(dev + (phase < 2 ? g.off_tp : g.off_tv));
        mg.nreq[q] = nreq;
        mg.begin[q + 1] = mg.begin[q] + nb;
    }
    *blocks = mg.begin[mg.n];
    return mg;
}

// One merged launch, timed per launch when profiling (kc 0: all buckets).
isvd_status chain_launch(isvd_engine* e, const std::vector<Group>& groups, const char* dev, int phase,
                         hipStream_t st) {
    int blocks = 0;
    const MultiGroup mg = chain_args(groups, dev, phase, &blocks);
    if (mg.n == 0) return ISVD_OK;
    LaunchRec rec{};
    if (e->profiling) {
        ST_TRY(next_event(e, &rec.b));
        ST_TRY(next_event(e, &rec.e));
        HIP_TRY(hipEventRecord(rec.b, st));
    }
    switch (phase) {
        case 0: k_proj_chain<1><<<blocks, kThreads, 0, st>>>(mg); break;
        case 1: k_proj_chain<2><<<blocks, kThreads, 0, st>>>(mg); break;
        case 2: k_core_chain<<<blocks, kSecCoreThreads, sizeof(double) * chain_core_lds(), st>>>(mg); break;
        case 4: k_rotv_chain<<<blocks + 1, kThreads, 0, st>>>(mg, e->chain_plan); break;
        default: k_rotu_chain<<<kChainUGrid, kThreads, 0, st>>>(mg, e->chain_plan); break;
    }
    HIP_TRY(hipGetLastError());
    if (e->profiling) {
        HIP_TRY(hipEventRecord(rec.e, st));
        rec.phase = phase;
        rec.kc = 0;
        rec.fp64 = 0;
        int nreq = 0;
        for (int q = 0; q < mg.n; ++q) nreq += mg.nreq[q];
        rec.nreq = nreq;
        rec.blocks = phase == 3 ? kChainUGrid : blocks;
        e->prof.push_back(rec);
    }
    return ISVD_OK;
}

// A merged tick: (upload,) projections, cores, V rotations, the U plan and
// the planned U rotations, all on `st`.
isvd_status chain_sequence(isvd_engine* e, const std::vector<Group>& groups, const char* host, char* dev,
                           size_t bytes, hipStream_t st, bool upload) {
    if (upload) {
        const size_t n16 = align_up(bytes, 16) / 16;
        if (n16 > 0)
            k_upload<<<(int)std::min<size_t>(cdiv(n16, 256), 64), 256, 0, st>>>(
                reinterpret_cast<const uint4*>(host), reinterpret_cast<uint4*>(dev), n16);
        HIP_TRY(hipGetLastError());
    }
    for (int phase : {0, 1, 2, 4, 3}) ST_TRY(chain_launch(e, groups, dev, phase, st));
    return ISVD_OK;
}

void free_tick_graph(TickGraph* tg) {
    for (int b = 0; b < kTickGraphBufs; ++b) {
        if (tg->done[b]) (void)hipEventSynchronize(tg->done[b]);
        if (tg->exec[b]) (void)hipGraphExecDestroy(tg->exec[b]);
        if (tg->graph[b]) (void)hipGraphDestroy(tg->graph[b]);
        if (tg->done[b]) (void)hipEventDestroy(tg->done[b]);
        if (tg->host[b]) (void)hipHostFree(tg->host[b]);
        if (tg->dev[b]) (void)hipFree(tg->dev[b]);
    }
    delete tg;
}

constexpr size_t kMaxTickGraphs = 4;

// A deferred-U tick of row appends as one replay of a captured graph (see
// TickGraph); the first tick of a request set captures it.
isvd_status run_groups_graph(isvd_engine* e, std::vector<Group>& groups, hipStream_t st, bool pipelined) {
    ST_TRY(ensure_lanes(e));
    const bool chain = chain_ok(e, groups);
    const size_t off = layout_groups(groups, chain);
    std::vector<int64_t> key;
    for (const Group& g : groups) {
        key.insert(key.end(), {(int64_t)g.kc, (int64_t)(g.fp64 * 2 + g.bf16), (int64_t)g.var, (int64_t)g.rows,
                               (int64_t)g.all.size(), (int64_t)g.proj.size(), (int64_t)g.rotU_cap});
        key.insert(key.end(), g.ids.begin(), g.ids.end());
    }
    if (chain) ST_TRY(ensure_chain_plan(e));
    TickGraph* tg = nullptr;
    for (TickGraph* c : e->tgraphs)
        if (c->key == key) tg = c;
    if (!tg) {
        if (!e->capture_st) HIP_TRY(hipStreamCreateWithFlags(&e->capture_st, hipStreamNonBlocking));
        if (e->tgraphs.size() >= kMaxTickGraphs) {
            auto it = std::min_element(e->tgraphs.begin(), e->tgraphs.end(),
                                       [](const TickGraph* a, const TickGraph* b) { return a->last_use < b->last_use; });
            free_tick_graph(*it);
            e->tgraphs.erase(it);
        }
        tg = new TickGraph();
        tg->key = key;
        tg->bytes = std::max<size_t>(off, 64);
        isvd_status rc = ISVD_OK;
        for (int b = 0; b < kTickGraphBufs && rc == ISVD_OK; ++b) {
            if (hipHostMalloc((void**)&tg->host[b], tg->bytes, hipHostMallocDefault) != hipSuccess ||
                hipMalloc((void**)&tg->dev[b], tg->bytes) != hipSuccess ||
                hipEventCreateWithFlags(&tg->done[b], hipEventDisableTiming) != hipSuccess) {
                rc = fail(ISVD_E_NOMEM, "captured tick buffers");
                break;
            }
            // U-rotation grids sized for the streams' capacity: the captured
            // grid serves every later tick of this request set
            for (Group& g : groups) g.grid_u = g.rotU_cap;
            if (hipStreamBeginCapture(e->capture_st, hipStreamCaptureModeRelaxed) != hipSuccess) {
                rc = fail(ISVD_E_DEVICE, "tick capture failed to begin");
                break;
            }
            rc = chain ? chain_sequence(e, groups, tg->host[b], tg->dev[b], off, e->capture_st, true)
                       : own_lane_sequence(e, groups, tg->host[b], tg->dev[b], off, e->capture_st);
            const hipError_t ce = hipStreamEndCapture(e->capture_st, &tg->graph[b]);
            for (Group& g : groups) g.grid_u = 0;
            if (rc == ISVD_OK && ce != hipSuccess) rc = fail(ISVD_E_DEVICE, "tick capture failed");
            if (rc == ISVD_OK && hipGraphInstantiate(&tg->exec[b], tg->graph[b], nullptr, nullptr, 0) != hipSuccess)
                rc = fail(ISVD_E_DEVICE, "tick graph instantiation failed");
        }
        if (rc != ISVD_OK) {
            free_tick_graph(tg);
            return rc;
        }
        e->tgraphs.push_back(tg);
    }
    tg->last_use = e->ticks;
    const int b = tg->next;
    tg->next = (tg->next + 1) % kTickGraphBufs;
    // the buffer's previous tick (kTickGraphBufs ticks ago) has read it
    if (tg->launched[b]) HIP_TRY(hipEventSynchronize(tg->done[b]));
    fill_groups(groups, tg->host[b]);
    if (e->ticks >= 2 && e->lane_ticks < 2) HIP_TRY(hipStreamWaitEvent(st, e->ev_tick_end[e->ticks & 1], 0));
    HIP_TRY(hipGraphLaunch(tg->exec[b], st));
    HIP_TRY(hipEventRecord(tg->done[b], st));
    tg->launched[b] = true;
    HIP_TRY(hipEventRecord(e->ev_tick_end[e->ticks & 1], st));
    e->ticks += 1;
    e->lane_ticks += 1;
    if (!pipelined) ST_TRY(join(e, st));   // rotation-lane work of earlier ticks
    return ISVD_OK;
}

isvd_status run_groups(isvd_engine* e, std::vector<Group>& groups, hipStream_t st, bool pipelined) {
    ST_TRY(ensure_lanes(e));
    const bool chain = chain_ok(e, groups);
    const size_t off = layout_groups(groups, chain);
    Slot* slot = nullptr;
    ST_TRY(acquire_slot(e, off, &slot));
    fill_groups(groups, slot->host);
    if (chain) {
        ST_TRY(ensure_chain_plan(e));
        if (e->ticks >= 2 && e->lane_ticks < 2) HIP_TRY(hipStreamWaitEvent(st, e->ev_tick_end[e->ticks & 1], 0));
        ST_TRY(upload_slot(slot, off, st));
        ST_TRY(chain_sequence(e, groups, slot->host, slot->dev, off, st, false));
        HIP_TRY(hipEventRecord(slot->ev, st));
        slot->used = true;
        HIP_TRY(hipEventRecord(e->ev_tick_end[e->ticks & 1], st));
        e->ticks += 1;
        e->lane_ticks += 1;
        if (!pipelined) ST_TRY(join(e, st));   // rotation-lane work of earlier ticks
        return ISVD_OK;
    }
    // With deferred U the U rotations are mostly skipped and run on the
    // group's own update lane after its V rotation; the whole tick then ends
    // on the caller's stream (no rotation lanes, two cross-stream waits).
    const bool own_lanes = e->defer_u;
    if (e->ticks >= 2 && !(own_lanes && e->lane_ticks >= 2))
        HIP_TRY(hipStreamWaitEvent(st, e->ev_tick_end[e->ticks & 1], 0));
    ST_TRY(upload_slot(slot, off, st));
    while (e->ev_core.size() < groups.size()) {
        hipEvent_t ev;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        e->ev_core.push_back(ev);
    }
    // Update lanes.  Explicit U: lane a for the 64-column bucket and wider,
    // lane b for the others (the U rotations dominate, on the rotation
    // lanes).  Deferred U: the cores dominate, and the 64-, 32- and 16/8-column
    // buckets get a lane each.
    auto lane_of = [&](const Group& g) -> int {
        if (g.kc >= 64) return 0;
        if (!own_lanes) return 1;
        return g.kc >= 32 ? 1 : 2;
    };
    constexpr int kLanes = 3;
    hipStream_t lanes[kLanes] = {e->lane_a, e->lane_b, e->lane_c};
    hipEvent_t lane_end[kLanes] = {e->ev_main, e->ev_b_end, e->ev_c_end};
    bool used[kLanes] = {false, false, false};
    bool use_rb = false;
    for (const Group& g : groups) {
        used[lane_of(g)] = true;
        use_rb = use_rb || g.kc < 64;
    }
    HIP_TRY(hipEventRecord(e->ev_fork, st));
    for (int l = 0; l < kLanes; ++l)
        if (used[l]) HIP_TRY(hipStreamWaitEvent(lanes[l], e->ev_fork, 0));
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const Group& g = groups[gi];
        hipStream_t ln = lanes[lane_of(g)];
        for (int phase = 0; phase < 3; ++phase) ST_TRY(launch_recorded(e, g, slot->dev, phase, ln));
        if (!own_lanes) HIP_TRY(hipEventRecord(e->ev_core[gi], ln));
        ST_TRY(launch_recorded(e, g, slot->dev, 4, ln));
        if (own_lanes) ST_TRY(launch_recorded(e, g, slot->dev, 3, ln));
    }
    // the update lanes read the caller's payloads (projections, V
    // rotations): the caller's stream passes the tick only after them, so a
    // payload freed in that stream's order is never overwritten while read
    for (int l = 0; l < kLanes; ++l)
        if (used[l]) {
            HIP_TRY(hipEventRecord(lane_end[l], lanes[l]));
            HIP_TRY(hipStreamWaitEvent(st, lane_end[l], 0));
        }
    if (own_lanes) {
        HIP_TRY(hipEventRecord(slot->ev, st));
        slot->used = true;
        HIP_TRY(hipEventRecord(e->ev_tick_end[e->ticks & 1], st));
        e->ticks += 1;
        e->lane_ticks += 1;
        if (!pipelined) ST_TRY(join(e, st));   // rotation-lane work of earlier ticks
        return ISVD_OK;
    }
    e->lane_ticks = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const Group& g = groups[gi];
        hipStream_t rl = g.kc >= 64 ? e->rot_lane : e->rot_lane_b;
        HIP_TRY(hipStreamWaitEvent(rl, e->ev_core[gi], 0));
        ST_TRY(launch_recorded(e, g, slot->dev, 3, rl));
    }
    // the tick ends on the rotation lane once every lane is through it
    for (int l = 0; l < kLanes; ++l)
        if (used[l]) HIP_TRY(hipStreamWaitEvent(e->rot_lane, lane_end[l], 0));
    if (use_rb) {
        HIP_TRY(hipEventRecord(e->ev_rot_b, e->rot_lane_b));
        HIP_TRY(hipStreamWaitEvent(e->rot_lane, e->ev_rot_b, 0));
    }
    HIP_TRY(hipEventRecord(slot->ev, e->rot_lane));
    slot->used = true;
    HIP_TRY(hipEventRecord(e->ev_tick_end[e->ticks & 1], e->rot_lane));
    e->ticks += 1;
    e->rot_pending = true;
    if (!pipelined) ST_TRY(join(e, st));
    return ISVD_OK;
}

// Tracker work of the angle-policy streams of one launch sequence.
Track make_track(const Stream& s, int kind, const void* payload) {
    const int par = (int)(s.t & 1);
    Track t{};
    t.hdr = s.hdr;
    t.rs = s.rs[par];
    t.kind = kind;
    t.scope = s.cfg.policy.angle_scope;
    t.tiles = kind == kCol ? (int)std::max<int64_t>(1, cdiv(s.m, kTrackRows)) : 0;
    t.kc = s.kc;
    t.Uref = s.Uref;
    t.U[0] = s.U[0];
    t.U[1] = s.U[1];
    t.QU = s.QU[par];
    t.p = s.p[par];
    t.S = s.S;
    t.payload = payload;
    t.M = s.TM;
    t.H = s.TH;
    t.part = s.TP;
    t.scr = s.TS;
    return t;
}

template <typename T>
isvd_status launch_tracks(const char* dev, size_t off_all, size_t off_col, size_t off_pre, int nall, int ncol,
                          int col_blocks, hipStream_t st) {
    const Track* all = reinterpret_cast<const Track*>(dev + off_all);
    if (ncol > 0)
        k_track_col<T><<<col_blocks, kTrackColThreads, 0, st>>>(reinterpret_cast<const Track*>(dev + off_col),
                                                       reinterpret_cast<const int*>(dev + off_pre), ncol);
    k_track<T><<<nall, kThreads, sizeof(double) * track_lds_doubles(), st>>>(all);
    k_theta_tracks<<<nall, WideShape::NT, sizeof(double) * theta_lds_doubles(), st>>>(all);
    HIP_TRY(hipGetLastError());
    return ISVD_OK;
}

// Runs after the update kernels on `st`: M, H through each update's rotation
// and theta_ref into the headers.  tracks[q] pairs with fp64[q].
isvd_status run_tracks(isvd_engine* e, const std::vector<Track>& tracks, const std::vector<char>& fp64,
                       hipStream_t st) {
    if (tracks.empty()) return ISVD_OK;
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<Track> all, col;
        for (size_t q = 0; q < tracks.size(); ++q)
            if ((fp64[q] != 0) == (pass == 1)) {
                all.push_back(tracks[q]);
                if (tracks[q].kind == kCol) col.push_back(tracks[q]);
            }
        if (all.empty()) continue;
        std::vector<int> pre(col.size() + 1, 0);
        for (size_t q = 0; q < col.size(); ++q) pre[q + 1] = pre[q] + col[q].tiles;
        size_t off = 0;
        auto take = [&](size_t b) {
            size_t o = off;
            off = align_up(off + b, 64);
            return o;
        };
        const size_t o_all = take(sizeof(Track) * all.size());
        const size_t o_col = take(sizeof(Track) * std::max<size_t>(1, col.size()));
        const size_t o_pre = take(sizeof(int) * pre.size());
        Slot* slot = nullptr;
        ST_TRY(acquire_slot(e, off, &slot));
        memcpy(slot->host + o_all, all.data(), sizeof(Track) * all.size());
        if (!col.empty()) memcpy(slot->host + o_col, col.data(), sizeof(Track) * col.size());
        memcpy(slot->host + o_pre, pre.data(), sizeof(int) * pre.size());
        ST_TRY(upload_slot(slot, off, st));
        if (pass == 1)
            ST_TRY(launch_tracks<double>(slot->dev, o_all, o_col, o_pre, (int)all.size(), (int)col.size(),
                                         pre.back(), st));
        else
            ST_TRY(launch_tracks<float>(slot->dev, o_all, o_col, o_pre, (int)all.size(), (int)col.size(),
                                        pre.back(), st));
        HIP_TRY(hipEventRecord(slot->ev, st));
        slot->used = true;
    }
    return ISVD_OK;
}

// ---------------------------------------------------------------- refresh
struct WsLayout {
    size_t X, Y, Zp, Gp, G, R, Racc, Rtmp, RinvT, QU, QV, Sr, flag, sweeps, fro, total;
};

WsLayout ws_layout(int64_t m, int64_t n, int b, int esz) {
    WsLayout w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const int64_t nchunk_tn = std::min<int64_t>(32, cdiv(m, kGemmK));
    const int64_t nchunk_g = gram_parts_max(std::max(m, n));
    w.X = take((size_t)esz * n * b);
    w.Y = take((size_t)esz * m * b);
    const int64_t ncb = cdiv(n, kTnCols);
    w.Zp = take(esz == 4 ? sizeof(float) * (size_t)tn_chunks(m, n) * ncb * kTnDump
                         : sizeof(double) * (size_t)nchunk_tn * n * b);
    w.Gp = take(sizeof(double) * (size_t)nchunk_g * gram_tiles(b) * 256);
    w.G = take(sizeof(double) * b * b);
    w.R = take(sizeof(double) * b * b);
    w.Racc = take(sizeof(double) * b * b);
    w.Rtmp = take(sizeof(double) * b * b);
    w.RinvT = take((size_t)esz * b * b);
    w.QU = take((size_t)esz * b * 128);
    w.QV = take((size_t)esz * b * 128);
    w.Sr = take(sizeof(double) * 128);
    w.flag = take(sizeof(int) * 4);
    w.sweeps = take(sizeof(int) * 4);
    w.fro = take(sizeof(double) * (size_t)cdiv(m, kFroRows));
    w.total = off;
    return w;
}

isvd_status ensure_ws(WsBuf& w, size_t bytes) {
    if (w.bytes >= bytes) return ISVD_OK;
    if (w.fixed) return fail(ISVD_E_NOMEM, "refresh workspace of %zu bytes exceeds the fixed %zu", bytes, w.bytes);
    if (w.p) {
        if (w.defer_free) {
            w.retired.push_back(w.p);
        } else {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(w.p));
        }
        w.p = nullptr;
        w.bytes = 0;
    }
    // some slack, so that streams of slowly growing size do not reallocate each time
    const size_t want = bytes + bytes / 4;
    if (hipMalloc((void**)&w.p, want) != hipSuccess) {
        w.p = nullptr;
        return fail(ISVD_E_NOMEM, "refresh workspace of %zu bytes", want);
    }
    w.bytes = want;
    return ISVD_OK;
}
isvd_status ensure_ws(isvd_engine* e, size_t bytes) { return ensure_ws(e->ws, bytes); }

void free_retired(WsBuf& w) {
    for (char* q : w.retired) (void)hipFree(q);
    w.retired.clear();
}

// deterministic values in [-1, 1) (autotuner inputs)
__global__ void k_fill_hash(float* x, int64_t n, uint32_t seed) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)e * 2654435761u ^ seed;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        x[e] = (float)((double)h * (2.0 / 4294967296.0) - 1.0);
    }
}

__global__ void k_set_header(DevHeader* hdr, int k, int ld, int flip, int bump_t) {
    if (threadIdx.x == 0) {
        hdr->k = k;
        hdr->ld = ld;
        if (flip) hdr->cur ^= 1;
        if (bump_t) hdr->t += 1;
    }
}

// Y = A X on the matrix cores (FP32); the kernels are specialised on the
// number of 16-column tiles of X
template <int RB>
void gemm_nn_rb(const float* A, int64_t lda, const float* X, float* Y, int ldy, int64_t m, int64_t n, int b,
                hipStream_t st) {
    const int grid = (int)cdiv(m, 64 * RB);
#define ISVD_NN(NB) k_gemm_nn_mfma<RB, NB><<<grid, kThreads, 0, st>>>(A, lda, X, Y, ldy, m, n, b)
    switch ((b + 15) / 16) {
        case 1: ISVD_NN(1); break;
        case 2: ISVD_NN(2); break;
        case 3: ISVD_NN(3); break;
        case 4: ISVD_NN(4); break;
        case 5: ISVD_NN(5); break;
        case 6: ISVD_NN(6); break;
        case 7: ISVD_NN(7); break;
        default: ISVD_NN(8); break;
    }
#undef ISVD_NN
}
// X is n x b with leading dimension b
void gemm_nn_f32(const float* A, int64_t lda, const float* X, float* Y, int ldy, int64_t m, int64_t n, int b,
                 hipStream_t st) {
    gemm_nn_rb<2>(A, lda, X, Y, ldy, m, n, b, st);
}
// partial dumps of Z = A^T Q on the matrix cores (FP32)
// Q is m x b with leading dimension b
void gemm_tn_f32(const float* A, int64_t lda, const float* Q, float* Zp, int64_t m, int64_t n, int b, int64_t nch,
                 hipStream_t st) {
    const dim3 grid((unsigned)cdiv(n, kTnCols), (unsigned)nch);
    const int64_t rpc = cdiv(m, nch);
#define ISVD_TN(NB) k_gemm_tn_mfma<NB><<<grid, kThreads, 0, st>>>(A, lda, Q, Zp, m, n, b, rpc)
    switch ((b + 15) / 16) {
        case 1: ISVD_TN(1); break;
        case 2: ISVD_TN(2); break;
        case 3: ISVD_TN(3); break;
        case 4: ISVD_TN(4); break;
        case 5: ISVD_TN(5); break;
        case 6: ISVD_TN(6); break;
        case 7: ISVD_TN(7); break;
        default: ISVD_TN(8); break;
    }
#undef ISVD_TN
}

// Y <- Q with Y = Q R: `passes` CholQR passes (2 = CholQR2, orthonormal to
// working precision; 1 leaves an orthogonality error of about kappa(Y) times
// the storage epsilon, which is all an intermediate block of the subspace
// iteration needs: only its span is used).
// With want_R, *R_out receives where the product of the passes' R factors is
// left (R_2 R_1 for two passes).
template <typename T>
isvd_status cholqr(char* ws, const WsLayout& w, T* Y, int64_t rows, int b, bool want_R, int passes,
                   hipStream_t st, const double** R_out = nullptr) {
    double* Gp = (double*)(ws + w.Gp);
    double* G = (double*)(ws + w.G);
    double* R = (double*)(ws + w.R);
    double* Racc = (double*)(ws + w.Racc);
    double* Rtmp = (double*)(ws + w.Rtmp);
    T* RinvT = (T*)(ws + w.RinvT);
    int* flag = (int*)(ws + w.flag);
    const int nchunk = (int)gram_parts(rows);
    for (int pass = 0; pass < passes; ++pass) {
        k_gram_mfma<T><<<nchunk, kThreads, 0, st>>>(Y, b, rows, b, gram_rpb(rows), Gp);
        k_gram_sum<<<(int)cdiv(gram_tiles(b) * 256, 32), 256, 0, st>>>(Gp, nchunk, b, G);
        // the first pass's R goes straight where the product needs it
        k_chol_inv<T><<<1, kCholThreads, 0, st>>>(G, b, want_R && pass == 0 ? Racc : R, RinvT, flag);
        if constexpr (sizeof(T) == 4) {
            if (b % 4 == 0)
                gemm_nn_f32(Y, b, RinvT, Y, b, rows, b, b, st);
            else
                k_rotate_plain<T, 128><<<(int)cdiv(rows, 16), kThreads, 0, st>>>(Y, b, Y, b, rows, b, RinvT);
        } else {
            k_rotate_plain<T, 128><<<(int)cdiv(rows, 16), kThreads, 0, st>>>(Y, b, Y, b, rows, b, RinvT);
        }
        if (want_R && pass == 1) k_small_gemm<<<(int)cdiv(b * b, 256), 256, 0, st>>>(R, Racc, Rtmp, b);
    }
    if (want_R && R_out) *R_out = passes >= 2 ? Rtmp : Racc;
    HIP_TRY(hipGetLastError());
    return ISVD_OK;
}

// Y = A X: matrix cores for FP32 storage, FP64 VALU tiles for FP64
template <typename T>
void gemm_nn(const T* A, int64_t lda, const T* X, T* Y, int64_t m, int64_t n, int b, hipStream_t st) {
    if constexpr (sizeof(T) == 4)
        gemm_nn_f32(A, lda, X, Y, b, m, n, b, st);
    else
        k_gemm_nn<T><<<(int)cdiv(m, kGemmRows), kThreads, 0, st>>>(A, lda, X, b, Y, b, m, n, b);
}

// Rank and block size of a refresh of the stream's current shape.
void refresh_block(const Stream& s, int* k_out, int* b_out) {
    const int64_t m = s.m, n = s.n;
    const int k = (int)std::min<int64_t>(s.k_target, std::min(m, n));
    const int os = s.cfg.oversample >= 0 ? s.cfg.oversample : std::max(8, k / 2);
    int b = (int)std::min<int64_t>(n, (int64_t)k + os);
    b = std::min(b, kMaxBlock);
    b = (int)std::min<int64_t>(b, m);
    *k_out = k;
    *b_out = b;
}

bool gram_form(const Stream& s, int b) { return b != s.n && s.n <= kGcfMaxN && s.cfg.refresh_iters < 0; }

// TruncatedSVD(A_t, k), in two steps so that a check of the error policy can
// compute it, look at its Ritz values, and commit it only if the policy fires.
struct RefreshPlan {
    int k = 0, b = 0, ldo = 0, cur = 0;
    int64_t m = 0, n = 0;
    WsLayout w{};
    int rounds = 0;          // Gram form: Rayleigh-Ritz rounds until the stopping rule held
    bool converged = true;   // Gram form: all k Ritz pairs met the residual tolerance
    // Gram form: the leading k Ritz values of G = A^T A (sigma^2, from exact
    // FP64 products), non-increasing; E_opt^2 = ||A||^2 minus the sum of the
    // first (model rank) of them.  Empty in the A form.
    std::vector<double> gram_theta;
};

// Row chunks of the Gram product: the grid (tiles x chunks) is sized to
// whole waves of two 256-thread blocks per compute unit (a partial last
// wave of blocks would idle most of the chip for a block's duration),
// chunks of at least 256 rows, at most 2048 partial tiles (256 MB).
constexpr int kXtyRows = 64;   // rows per block of the small cross products X^T Y
int ata_chunks(int64_t m, int ntile) {
    const int64_t cap = 2 * 256;
    int best = 1;
    double best_cost = 1e300;
    for (int c = 1; c <= 64; ++c) {
        if (c > 1 && (cdiv(m, c) < 256 || (int64_t)ntile * c > 2048)) break;
        const int64_t blocks = (int64_t)ntile * c;
        const double waves = (double)cdiv(blocks, cap);
        // time ~ whole waves of blocks, each 1 / c of the rows; a small
        // charge per chunk for its partial tile
        const double cost = waves / c + 0.0005 * c;
        if (cost < best_cost) {
            best_cost = cost;
            best = c;
        }
    }
    return best;
}

// Workspace of the Gram-form refresh, placed after the A-form layout of
// its final step.
struct GcfLayout {
    size_t G, Gp, X, Xn, W, Wn, Y0, Y1, Y2, L, Hp, C, H, R, Rinv, P, PU, sig, theta, res, flag, sweeps, total;
    int ldg = 0, nchunk = 1, nxty = 1;
};

GcfLayout gcf_layout(int64_t m, int64_t n, size_t base, size_t cap = SIZE_MAX, int nchunk = 0) {
    if (nchunk == 0) {
        // fewer row chunks (smaller partial buffer) when the workspace is capped
        for (int c = ata_chunks(m, ata_tiles(n)); c >= 1; --c) {
            const GcfLayout t = gcf_layout(m, n, base, SIZE_MAX, c);
            if (t.total <= cap || c == 1) return t;
        }
    }
    GcfLayout g{};
    size_t off = align_up(base, 256);
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    g.ldg = (int)round64(n);
    const int ntile = ata_tiles(n);
    g.nchunk = nchunk;
    g.nxty = (int)cdiv(g.ldg, kXtyRows);
    const size_t blk = sizeof(double) * (size_t)g.ldg * kMaxBlock;
    const size_t sq = sizeof(double) * kMaxBlock * kMaxBlock;
    g.G = take(sizeof(double) * (size_t)g.ldg * g.ldg);
    g.Gp = take(sizeof(double) * (size_t)g.nchunk * ntile * kAtaTile * kAtaTile);
    g.X = take(blk);
    g.Xn = take(blk);
    g.W = take(blk);
    g.Wn = take(blk);
    g.Y0 = take(blk);
    g.Y1 = take(blk);
    g.Y2 = take(blk);
    g.L = take(blk);
    g.Hp = take(sq * (size_t)std::max<int64_t>(g.nxty, gram_parts_max(g.ldg)));
    g.C = take(sq);
    g.H = take(sq);
    g.R = take(sq);
    g.Rinv = take(sq);
    g.P = take(sq);
    g.PU = take(sq);
    g.sig = take(sizeof(double) * kMaxBlock);
    g.theta = take(sizeof(double) * kMaxBlock);
    g.res = take(sizeof(double) * kMaxBlock);
    g.flag = take(sizeof(int) * 4);
    g.sweeps = take(sizeof(int) * 4);
    g.total = off;
    return g;
}

// Y (rows x w, FP64, leading dimension w) <- CholQR2(Y): Gram on the FP64
// matrix cores, Cholesky and R^{-1} in one block, Y R^{-1}, twice.  Zero
// columns stay zero (their pivots are dropped).
isvd_status gcf_orth(char* ws, const GcfLayout& g, double* Y, int64_t rows, int w, hipStream_t st) {
    double* Gp = (double*)(ws + g.Hp);
    double* Hg = (double*)(ws + g.H);
    double* R = (double*)(ws + g.R);
    double* Rinv = (double*)(ws + g.Rinv);
    int* flag = (int*)(ws + g.flag);
    const int nchunk = (int)gram_parts(rows);
    for (int pass = 0; pass < 2; ++pass) {
        k_gram_mfma<double><<<nchunk, kThreads, 0, st>>>(Y, w, rows, w, gram_rpb(rows), Gp);
        k_gram_sum<<<(int)cdiv(gram_tiles(w) * 256, 32), 256, 0, st>>>(Gp, nchunk, w, Hg);
        k_chol_inv<double><<<1, kCholThreads, 0, st>>>(Hg, w, R, Rinv, flag);
        k_rotate_plain<double, 128><<<(int)cdiv(rows, 16), kThreads, 0, st>>>(Y, w, Y, w, rows, w, Rinv);
    }
    HIP_TRY(hipGetLastError());
    return ISVD_OK;
}

// FP64 storage iterates down to rounding level (the stagnation clause of the
// stopping rule ends it there); FP32 storage, whose factors carry 2^-24
// rounding anyway, stops at 1e-10 theta_1.
double gcf_default_tol(const Stream& s) {
    if (s.cfg.refresh_tol > 0.0) return s.cfg.refresh_tol;
    return s.esz == 8 ? 1e-16 : 1e-10;
}

constexpr int kGcfMaxRounds = 40;
constexpr double kGcfBig = 16.0;       // a Ritz value this far above the cut is deflated once converged
constexpr double kGcfLockTol = 1e-14;  // ... to this residual (relative to theta_1) at the least
constexpr int kGcfMaxDegree = 24;
constexpr double kGcfGrowth = 1e6;   // largest growth of an active Ritz value per filter

// Gram-form TruncatedSVD (see isvd_gcf.h): right vectors by Chebyshev-
// filtered subspace iteration on G = A^T A with locking, until the leading k
// Ritz residuals are at most tol * theta_1; then Y = A L, CholQR2 and the
// Rayleigh-Ritz SVD of R as in the A form, with block k.  The host reads the
// Ritz values and residuals once per round to lock, stop and pick the filter.
template <typename T>
isvd_status refresh_compute_gcf(isvd_engine* e, Stream& s, bool init, hipStream_t st, RefreshPlan* plan,
                                const DevHeader& h, int k, int b, WsBuf& wb, int* sweeps_dev) {
    const int64_t m = s.m, n = s.n;
    const WsLayout w = ws_layout(m, n, b, (int)sizeof(T));
    const GcfLayout g = gcf_layout(m, n, w.total, wb.fixed ? wb.bytes : SIZE_MAX);
    ST_TRY(ensure_ws(wb, g.total));
    char* ws = wb.p;
    const T* A = (const T*)s.A;
    const int64_t lda = lda_of(s.cfg);
    const int ldg = g.ldg;
    double* G = (double*)(ws + g.G);
    double* X = (double*)(ws + g.X);
    double* Xn = (double*)(ws + g.Xn);
    double* W = (double*)(ws + g.W);
    double* Wn = (double*)(ws + g.Wn);
    double* Yb[3] = {(double*)(ws + g.Y0), (double*)(ws + g.Y1), (double*)(ws + g.Y2)};
    double* L = (double*)(ws + g.L);
    double* Hp = (double*)(ws + g.Hp);
    double* C = (double*)(ws + g.C);
    double* H = (double*)(ws + g.H);
    double* R = (double*)(ws + g.R);
    double* Rinv = (double*)(ws + g.Rinv);
    double* P = (double*)(ws + g.P);
    double* PU = (double*)(ws + g.PU);
    double* sig = (double*)(ws + g.sig);
    double* theta = (double*)(ws + g.theta);
    double* res = (double*)(ws + g.res);
    int* flag = (int*)(ws + g.flag);
    int* gsweeps = (int*)(ws + g.sweeps);
    const int kL = kMaxBlock;
    const double tol = gcf_default_tol(s);
    // G = A^T A
    const int ntile = ata_tiles(n);
    k_ata_mfma<T><<<dim3((unsigned)ntile, (unsigned)g.nchunk), kThreads, 0, st>>>(A, lda, m, n, cdiv(m, g.nchunk),
                                                                                   (double*)(ws + g.Gp));
    k_ata_sum<<<(int)cdiv((int64_t)ldg * ldg, 256), 256, 0, st>>>((const double*)(ws + g.Gp), g.nchunk, n, ldg, G);
    // start block
    int ba = b, wa = (int)round16(b);
    const int kw = init ? 0 : std::min(h.k, b);
    k_gcf_start<T><<<(int)cdiv((int64_t)ldg * wa, 256), 256, 0, st>>>(
        X, wa, n, ldg, b, (const T*)s.V[init ? 0 : h.cur], init ? 4 : h.ld, kw, 0x5eedull + (uint64_t)s.t);
    ST_TRY(gcf_orth(ws, g, X, ldg, wa, st));
    std::vector<double> hbuf(2 * kMaxBlock + 1);
    int nlk = 0, rounds = 0, nl_last = 0;
    double th1 = 0.0, prev_rmax = HUGE_VAL;
    bool converged = false;
    const double lock_tol = std::max(tol, kGcfLockTol);
    std::vector<double> locked_theta;
    std::vector<double> gram_theta;
    for (;;) {
        ++rounds;
        // Rayleigh-Ritz on the active block
        k_symm_cheb<<<dim3((unsigned)(ldg / 16), (unsigned)cdiv(wa, 32)), kThreads, 0, st>>>(G, ldg, X, nullptr, W,
                                                                                            wa, wa, 1.0, 0.0, 0.0);
        k_xty_partial<<<g.nxty, kThreads, 0, st>>>(X, wa, wa, W, wa, wa, ldg, kXtyRows, Hp);
        k_sum_sym<<<(int)cdiv(wa * wa, 256), 256, 0, st>>>(Hp, g.nxty, wa, H);
        k_chol_inv<double><<<1, kCholThreads, 0, st>>>(H, wa, R, Rinv, flag);
        // right vectors P of R (the eigenvectors of H) from the rotated columns
        // of R^T, without accumulating the rotations: their orthogonality loss,
        // about b eps64 (theta_1 / theta_j)^(1/2), stays near rounding level
        k_svd_small_noj<double><<<1, RRShape::NT, sizeof(double) * svd_noj_lds_doubles(), st>>>(R, wa, wa, sig,
                                                                                               PU, P, wa, gsweeps);
        k_rotate_plain<double, 128><<<ldg / 16, kThreads, 0, st>>>(X, wa, Xn, wa, ldg, wa, P);
        k_rotate_plain<double, 128><<<ldg / 16, kThreads, 0, st>>>(W, wa, Wn, wa, ldg, wa, P);
        std::swap(X, Xn);
        std::swap(W, Wn);
        k_ritz_res<<<wa, kThreads, 0, st>>>(W, X, wa, ldg, sig, theta, res);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(hbuf.data(), theta, sizeof(double) * wa, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hbuf.data() + kMaxBlock, res, sizeof(double) * wa, hipMemcpyDeviceToHost, st));
        int rr_sweeps = 0;
        HIP_TRY(hipMemcpyAsync(&rr_sweeps, gsweeps, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (rr_sweeps < 0) return fail(ISVD_E_CONVERGE, "Gram-form Rayleigh-Ritz Jacobi did not converge");
        const double* hth = hbuf.data();
        const double* hres = hbuf.data() + kMaxBlock;
        if (rounds == 1) th1 = hth[0];
        if (!(th1 > 0.0)) {
            // A = 0: every Ritz value is zero; the block is as good as any
            th1 = 1.0;
        }
        // stopping rule: the leading k pairs still in the active block meet
        // the tolerance, or their largest residual stopped falling (halving
        // per round) within 1e3 of it: rounding level
        double rmax = 0.0;
        for (int i = 0; i < k - nlk; ++i) rmax = std::max(rmax, hres[i]);
        rmax /= th1;
        const bool conv = rmax <= tol || (rmax <= 1e3 * tol && rmax > 0.5 * prev_rmax);
        prev_rmax = rmax;
        // deflate the converged pairs far above the cut (the factor directions):
        // they would otherwise limit the filter degree; pairs inside the bulk
        // stay active, so they keep improving until the whole set stops
        const double cut = hth[ba - 1];
        int nl = 0;
        while (nl < ba && nlk + nl < k && hres[nl] <= lock_tol * th1 && hth[nl] >= kGcfBig * cut) ++nl;
        if (conv || nlk + nl >= k || rounds >= kGcfMaxRounds) {
            gram_theta.assign(locked_theta.begin(), locked_theta.end());
            for (int i = 0; i < k - nlk; ++i) gram_theta.push_back(hth[i]);
            std::sort(gram_theta.begin(), gram_theta.end(), std::greater<double>());
        }
        for (int i = 0; i < nl; ++i) locked_theta.push_back(hth[i]);
        if (nl > 0) {
            k_copy2d<double, double><<<(int)cdiv((int64_t)ldg * nl, 256), 256, 0, st>>>(X, wa, L + nlk, kL, ldg, nl);
            const int nt16 = ldg / 16;
            k_deflate<<<nt16 * (nt16 + 1) / 2, kThreads, 0, st>>>(G, ldg, X, W, wa, nl, theta);
            nlk += nl;
        }
        nl_last = nl;
        if (conv || nlk >= k) {
            converged = true;
            break;
        }
        if (rounds >= kGcfMaxRounds) break;
        const double top = hth[nl];
        if (nl > 0) {
            // drop the locked columns, then refill the block with fresh ones
            const int keep = ba - nl;
            const int target = (int)std::max<int64_t>(keep, std::min<int64_t>(b, n - nlk));
            const int wn = (int)round16(target);
            k_take_cols<<<(int)cdiv((int64_t)ldg * wn, 256), 256, 0, st>>>(X, wa, nl, keep, Xn, wn, ldg);
            std::swap(X, Xn);
            if (target > keep)
                k_gcf_fill<<<(int)cdiv(n * (target - keep), 256), 256, 0, st>>>(
                    X, wn, n, keep, target, 0x5eedull + (uint64_t)s.t + 0x1000ull * (uint64_t)rounds);
            ba = target;
            wa = wn;
        }
        // Chebyshev filter on [0, cut]
        double alpha1, beta1, alpha2, beta2;
        int d;
        if (cut > 1e-14 * th1) {
            const double ec = 0.5 * cut;
            const double xt = 2.0 * top / cut - 1.0;
            d = xt > 1.0 + 1e-12 ? (int)std::floor(std::acosh(kGcfGrowth) / std::acosh(xt)) : kGcfMaxDegree;
            d = std::max(1, std::min(kGcfMaxDegree, d));
            alpha1 = 1.0 / ec;
            beta1 = -1.0;
            alpha2 = 2.0 / ec;
            beta2 = -2.0;
        } else {
            // the active block reaches the null space of A: plain power steps
            d = 1;
            alpha1 = top > 0.0 ? 1.0 / top : 1.0;
            beta1 = 0.0;
            alpha2 = beta2 = 0.0;
        }
        const dim3 grid((unsigned)(ldg / 16), (unsigned)cdiv(wa, 32));
        double* y0 = X;
        double* y1 = Yb[0];
        k_symm_cheb<<<grid, kThreads, 0, st>>>(G, ldg, y0, nullptr, y1, wa, wa, alpha1, beta1, 0.0);
        int nxt = 1;
        for (int j = 2; j <= d; ++j) {
            double* y2 = (y0 == X) ? Yb[nxt] : y0;
            if (y0 == X) nxt = 2;
            k_symm_cheb<<<grid, kThreads, 0, st>>>(G, ldg, y1, y0, y2, wa, wa, alpha2, beta2, -1.0);
            y0 = y1;
            y1 = y2;
        }
        // remove what the filter left of the locked directions (twice), then CholQR2
        for (int pass = 0; pass < 2 && nlk > 0; ++pass) {
            k_xty_partial<<<g.nxty, kThreads, 0, st>>>(L, kL, nlk, y1, wa, wa, ldg, kXtyRows, Hp);
            k_sum_parts<double><<<(int)cdiv(nlk * wa, 256), 256, 0, st>>>(Hp, g.nxty, (int64_t)nlk * wa,
                                                                          (int64_t)nlk * wa, C);
            k_sub_lc<<<(int)cdiv((int64_t)ldg * wa, 256), 256, 0, st>>>(y1, wa, wa, L, kL, nlk, C, ldg);
        }
        ST_TRY(gcf_orth(ws, g, y1, ldg, wa, st));
        if (y1 != X) {
            // the filtered block becomes X (X's buffer is one of the three)
            std::swap(X, (y1 == Yb[0] ? Yb[0] : (y1 == Yb[1] ? Yb[1] : Yb[2])));
        }
    }
    // Final step in A form on the whole block: the locked vectors and the
    // leading remaining active ones (b columns, orthonormal).  The Rayleigh-
    // Ritz SVD of R resolves the directions near the cut at the accuracy of
    // A itself, where G = A^T A, whose rounding is relative to sigma_1^2, can
    // only resolve them to about eps64 sigma_1^2 / (sigma_k (sigma_k -
    // sigma_k+1)) in angle.
    T* Xf = (T*)(ws + w.X);
    T* Y = (T*)(ws + w.Y);
    if (nlk > 0) k_copy2d<double, T><<<(int)cdiv(n * nlk, 256), 256, 0, st>>>(L, kL, Xf, b, n, nlk);
    k_copy2d<double, T><<<(int)cdiv(n * (b - nlk), 256), 256, 0, st>>>(X + nl_last, wa, Xf + nlk, b, n, b - nlk);
    k_start_flags<<<1, 64, 0, st>>>((int*)(ws + w.flag));
    gemm_nn<T>(A, lda, Xf, Y, m, n, b, st);
    const double* Rfin = nullptr;
    ST_TRY(cholqr<T>(ws, w, Y, m, b, true, 2, st, &Rfin));
    const int ldo = round4(k);
    // Rayleigh-Ritz SVD of R without accumulated rotations (an order-129
    // Jacobi with its rotations does not fit in LDS); the vectors' loss of
    // orthogonality, about b eps64 sigma_1 / sigma_j, is far below the FP32
    // rounding and within the FP64 bars for the kept triplets
    k_svd_small_noj<T><<<1, RRShape::NT, sizeof(double) * svd_noj_lds_doubles(), st>>>(
        Rfin, b, k, (double*)(ws + w.Sr), (T*)(ws + w.QU), (T*)(ws + w.QV), ldo,
        sweeps_dev ? sweeps_dev : (int*)(ws + w.sweeps));
    HIP_TRY(hipGetLastError());
    plan->k = k;
    plan->b = b;
    plan->ldo = ldo;
    plan->cur = init ? 0 : h.cur;
    plan->m = m;
    plan->n = n;
    plan->w = w;
    plan->rounds = rounds;
    plan->converged = converged;
    plan->gram_theta = gram_theta;
    return ISVD_OK;
}

// Block subspace iteration up to the Rayleigh-Ritz SVD: Ritz values in ws.Sr,
// left / right rotations of the block in ws.QU / ws.QV, block bases in
// ws.Y (Q_Y) and ws.X.  Nothing of the stream changes.
template <typename T>
isvd_status refresh_compute(isvd_engine* e, Stream& s, bool init, hipStream_t st, RefreshPlan* plan,
                            const DevHeader* known = nullptr, int* sweeps_dev = nullptr, WsBuf* wk = nullptr) {
    WsBuf& wb = wk ? *wk : e->ws;
    DevHeader h{};
    if (!init && known) {
        h = *known;
    } else if (!init) {
        HIP_TRY(hipMemcpyAsync(&h, s.hdr, sizeof(DevHeader), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    const int64_t m = s.m, n = s.n;
    int k = 0, b = 0;
    refresh_block(s, &k, &b);
    if (b < k) return fail(ISVD_E_INVAL, "refresh block %d smaller than rank %d", b, k);
    const bool exact = (b == n);
    if (gram_form(s, b))
        return refresh_compute_gcf<T>(e, s, init, st, plan, h, k, b, wb, sweeps_dev);
    const int iters = exact ? 0 : s.cfg.refresh_iters >= 0 ? s.cfg.refresh_iters : (init ? 8 : 3);
    WsLayout w = ws_layout(m, n, b, (int)sizeof(T));
    ST_TRY(ensure_ws(wb, w.total));
    char* ws = wb.p;
    T* X = (T*)(ws + w.X);
    T* Y = (T*)(ws + w.Y);
    double* Zp = (double*)(ws + w.Zp);
    const T* A = (const T*)s.A;
    const int64_t lda = lda_of(s.cfg);
    const int cur = init ? 0 : h.cur;
    const int kw = init ? 0 : std::min(h.k, b);
    k_start_block<T><<<(int)cdiv(n * b, 256), 256, 0, st>>>(X, b, n, b, (const T*)s.V[cur], init ? 4 : h.ld, kw,
                                                           0x5eedull + (uint64_t)s.t, exact ? 1 : 0,
                                                           (int*)(ws + w.flag));
    if (!exact) ST_TRY(cholqr<T>(ws, w, X, n, b, false, iters > 0 ? 1 : 2, st));
    const int64_t nchunk = std::min<int64_t>(32, cdiv(m, kGemmK));
    const int64_t rpc = cdiv(m, nchunk);
    for (int it = 0; it < iters; ++it) {
        gemm_nn<T>(A, lda, X, Y, m, n, b, st);
        ST_TRY(cholqr<T>(ws, w, Y, m, b, false, 1, st));
        if constexpr (sizeof(T) == 4) {
            const int64_t ncb = cdiv(n, kTnCols), nch = tn_chunks(m, n), per = ncb * kTnDump;
            gemm_tn_f32(A, lda, Y, (float*)Zp, m, n, b, nch, st);
            k_tn_sum<<<(int)cdiv(per, 256), 256, 0, st>>>((const float*)Zp, (int)nch, per, n, b, X, b);
        } else {
            dim3 grid((unsigned)cdiv(n, 64), (unsigned)nchunk);
            k_gemm_tn_partial<T><<<grid, kThreads, 0, st>>>(A, lda, Y, b, Zp, m, n, b, rpc);
            k_sum_parts<T><<<(int)cdiv(n * b, 256), 256, 0, st>>>(Zp, (int)nchunk, n * b, n * b, X);
        }
        ST_TRY(cholqr<T>(ws, w, X, n, b, false, it + 1 == iters ? 2 : 1, st));
    }
    gemm_nn<T>(A, lda, X, Y, m, n, b, st);
    const double* Rfin = nullptr;
    ST_TRY(cholqr<T>(ws, w, Y, m, b, true, 2, st, &Rfin));
    const int ldo = round4(k);
    k_svd_small_noj<T><<<1, RRShape::NT, sizeof(double) * svd_noj_lds_doubles(), st>>>(
        Rfin, b, k, (double*)(ws + w.Sr), (T*)(ws + w.QU), (T*)(ws + w.QV), ldo,
        sweeps_dev ? sweeps_dev : (int*)(ws + w.sweeps));
    HIP_TRY(hipGetLastError());
    plan->k = k;
    plan->b = b;
    plan->ldo = ldo;
    plan->cur = cur;
    plan->m = m;
    plan->n = n;
    plan->w = w;
    return ISVD_OK;
}

// Header after a refresh: the rank is the number of Ritz values above
// kRankTol sigma_1 (at least one), the numerical rank of A when it is below
// k: directions past it are arbitrary at FP64 rounding and are left out, and
// appends bring the rank back.  Also copies the Ritz values Sr into the
// stream's S.
constexpr double kRankTol = 1e-12;
__device__ inline void commit_header_body(DevHeader* hdr, double* S_out, const double* S, int k, int ld) {
    for (int j = threadIdx.x; j < k; j += blockDim.x) S_out[j] = S[j];
    if (threadIdx.x == 0) {
        const double cut = kRankTol * S[0];
        int kr = 1;
        while (kr < k && S[kr] > cut) ++kr;
        double s2 = 0.0;
        for (int j = 0; j < kr; ++j) s2 += S[j] * S[j];
        hdr->k = kr;
        hdr->ld = ld;
        hdr->cur ^= 1;
        hdr->sigma2 = s2;
        hdr->sigma_last = S[kr - 1];
    }
}
__global__ void k_commit_header(DevHeader* hdr, double* S_out, const double* S, int k, int ld) {
    commit_header_body(hdr, S_out, S, k, ld);
}

// The commit of a segmented refresh batch, one block (256 threads) per
// stream: the header (as k_commit_header), W and W^-1 of deferred-U streams
// back to I (as k_defer_reset), the reference trackers of angle streams reset
// (as k_track_reset), in that order.
struct SjCommit {
    DevHeader* hdr;
    double* S_out;
    const double* S;
    double* W[4];
    double* TM;
    double* TH;
    int k, ld, kcw, kct;
};
__global__ void __launch_bounds__(256) k_seg_commit(const SjCommit* __restrict__ jobs) {
    const SjCommit a = jobs[blockIdx.x];
    commit_header_body(a.hdr, a.S_out, a.S, a.k, a.ld);
    __syncthreads();
    if (a.W[0]) defer_reset_body(a.hdr, a.W[0], a.W[1], a.W[2], a.W[3], a.kcw, 0);
    __syncthreads();
    track_reset_body(a.hdr, a.TM, a.TH, a.kct);
}

__global__ void k_sigma_trackers(DevHeader* hdr, const double* S, int k) {
    if (threadIdx.x == 0) {
        double s2 = 0.0;
        for (int j = 0; j < k; ++j) s2 += S[j] * S[j];
        hdr->sigma2 = s2;
        hdr->sigma_last = k > 0 ? S[k - 1] : 0.0;
    }
}

// Adaptive rank: drop the last triplet (columns past k are ignored by every kernel).
__device__ inline void shrink_one(DevHeader* hdr, const double* S) {
    if (hdr->k > 1) {
        const int k = hdr->k - 1;
        hdr->k = k;
        hdr->sigma2 -= S[k] * S[k];
        hdr->sigma_last = S[k - 1];
    }
}
__global__ void k_shrink(DevHeader* hdr, const double* S) {
    if (threadIdx.x == 0) shrink_one(hdr, S);
}
// the shrinks of one tick, passed by value (thread i: stream i)
constexpr int kShrinkBatch = 224;
struct ShrinkList {
    int n;
    DevHeader* hdr[kShrinkBatch];
    const double* S[kShrinkBatch];
};
__global__ void k_shrink_many(ShrinkList L) {
    if ((int)threadIdx.x < L.n) shrink_one(L.hdr[threadIdx.x], L.S[threadIdx.x]);
}

isvd_status ensure_mws(isvd_engine* e, size_t bytes);

// M = U_ref^T U[0:m_ref, :] and H = U[0:m_ref, :]^T U[0:m_ref, :] formed
// directly (one pass over U_ref and U's reference rows), written with row
// stride ldo into M / H (device, when not null); with theta != nullptr also
// theta_ref into *theta (host; waits for the device).  Used by exact metrics
// and after a refresh that keeps the old reference.
template <typename T>
isvd_status direct_trackers_t(isvd_engine* e, Stream& s, hipStream_t st, double* theta, double* M, double* H,
                              int ldo) {
    DevHeader h{};
    HIP_TRY(hipMemcpyAsync(&h, s.hdr, sizeof(h), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int k = h.k, kref = h.ref_k;
    const int64_t mref = std::min<int64_t>(h.ref_m, h.m);
    const int64_t chunk = 1024;
    const int64_t nch = std::max<int64_t>(1, cdiv(mref, chunk));
    const size_t need = sizeof(double) * (size_t)(nch * (kref * k + k * k) + kref * k + 2 * k * k + 16);
    ST_TRY(ensure_mws(e, need));
    double* cp = (double*)e->mws;
    double* hp = cp + nch * kref * k;
    double* Md = hp + nch * k * k;
    double* Hd = Md + kref * k;
    const T* U = (const T*)s.U[h.cur];
    k_cross_partial<T><<<(int)nch, kThreads, 0, st>>>((const T*)s.Uref, h.ref_ld, kref, U, h.ld, k, mref, chunk, cp);
    k_cross_partial<T><<<(int)nch, kThreads, 0, st>>>(U, h.ld, k, U, h.ld, k, mref, chunk, hp);
    k_sum_parts<double><<<(int)cdiv(kref * k, 256), 256, 0, st>>>(cp, (int)nch, (int64_t)kref * k,
                                                                 (int64_t)kref * k, Md);
    k_sum_parts<double><<<(int)cdiv(k * k, 256), 256, 0, st>>>(hp, (int)nch, (int64_t)k * k, (int64_t)k * k, Hd);
    double* thd = Hd + k * k;
    double* Rg = thd + 8;   // j x j Cholesky factor of the theta kernel
    if (theta)
        k_theta_direct<<<1, WideShape::NT, sizeof(double) * theta_lds_doubles(), st>>>(
            Md, Hd, k, kref, s.S, s.cfg.policy.kind == ISVD_POL_ANGLE ? s.cfg.policy.angle_scope : 0, thd, Rg);
    if (M) {
        k_copy2d<double, double><<<(int)cdiv(kref * k, 256), 256, 0, st>>>(Md, k, M, ldo, kref, k);
        k_copy2d<double, double><<<(int)cdiv(k * k, 256), 256, 0, st>>>(Hd, k, H, ldo, k, k);
    }
    HIP_TRY(hipGetLastError());
    if (theta) {
        HIP_TRY(hipMemcpyAsync(theta, thd, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return ISVD_OK;
}

isvd_status direct_trackers(isvd_engine* e, Stream& s, hipStream_t st, double* theta, double* M, double* H, int ldo) {
    return s.esz == 8 ? direct_trackers_t<double>(e, s, st, theta, M, H, ldo)
                      : direct_trackers_t<float>(e, s, st, theta, M, H, ldo);
}

// Install the computed TruncatedSVD as the stream's state.
// sweeps_deferred: the Rayleigh-Ritz sweep count went to a caller's slot,
// which the caller checks (no wait here).
template <typename T>
isvd_status refresh_commit(isvd_engine* e, Stream& s, const RefreshPlan& plan, bool store_ref, hipStream_t st,
                           bool sweeps_deferred = false, WsBuf* wk = nullptr) {
    char* ws = wk ? wk->p : e->ws.p;
    const WsLayout& w = plan.w;
    const int nxt = plan.cur ^ 1;
    // U = Q_Y W (also into U_ref when the reference is stored), V = X H
    k_rotate_plain<T, 128, true><<<(int)cdiv(plan.m, 16), kThreads, 0, st>>>(
        (T*)(ws + w.Y), plan.b, (T*)s.U[nxt], plan.ldo, plan.m, plan.b, (T*)(ws + w.QU),
        store_ref ? (T*)s.Uref : nullptr);
    k_rotate_plain<T, 128, true><<<(int)cdiv(plan.n, 16), kThreads, 0, st>>>((T*)(ws + w.X), plan.b, (T*)s.V[nxt],
                                                                      plan.ldo, plan.n, plan.b, (T*)(ws + w.QV));
    k_commit_header<<<1, 64, 0, st>>>(s.hdr, s.S, (const double*)(ws + w.Sr), plan.k, plan.ldo);
    ST_TRY(defer_after_refresh(s, st));
    if (store_ref) {
        k_track_reset<<<1, kThreads, 0, st>>>(s.hdr, s.TM, s.TH, s.kc);
    } else if (s.TM) {
        ST_TRY(direct_trackers(e, s, st, nullptr, s.TM, s.TH, s.kc));
    }
    HIP_TRY(hipGetLastError());
    s.k_target = plan.k;
    if (sweeps_deferred) return ISVD_OK;
    int sweeps = 0;
    HIP_TRY(hipMemcpyAsync(&sweeps, ws + w.sweeps, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (sweeps < 0) return fail(ISVD_E_CONVERGE, "Rayleigh-Ritz Jacobi did not converge");
    return ISVD_OK;
}

// known: the stream's device header when the caller has it (saves a wait);
// sweeps_dev: device slot for the Rayleigh-Ritz sweep count, which the
// caller checks after the stream has run (without it this call waits).
isvd_status do_refresh(isvd_engine* e, Stream& s, bool init, bool store_ref, hipStream_t st,
                       const RefreshPlan* computed = nullptr, const DevHeader* known = nullptr,
                       int* sweeps_dev = nullptr, WsBuf* wk = nullptr) {
    HIP_TRY(hipEventRecord(s.ev_r0, st));
    RefreshPlan plan;
    isvd_status rc = ISVD_OK;
    if (computed) {
        plan = *computed;
    } else {
        rc = s.esz == 8 ? refresh_compute<double>(e, s, init, st, &plan, known, sweeps_dev, wk)
                        : refresh_compute<float>(e, s, init, st, &plan, known, sweeps_dev, wk);
        if (rc != ISVD_OK) return rc;
    }
    const bool deferred = sweeps_dev != nullptr && computed == nullptr;
    s.refresh_rounds = plan.rounds;
    s.refresh_converged = plan.converged;
    rc = s.esz == 8 ? refresh_commit<double>(e, s, plan, store_ref, st, deferred, wk)
                    : refresh_commit<float>(e, s, plan, store_ref, st, deferred, wk);
    if (rc != ISVD_OK) return rc;
    HIP_TRY(hipEventRecord(s.ev_r1, st));
    s.have_refresh_time = true;
    if (!init) {
        s.n_refresh += 1;
        s.t_last = s.t;
    }
    s.drift_acc = 0.0;
    return ISVD_OK;
}

// ------------------------------------------------------------ exact metrics
isvd_status ensure_mws(isvd_engine* e, size_t bytes) {
    if (e->mws_bytes >= bytes) return ISVD_OK;
    if (e->mws) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(e->mws));
        e->mws = nullptr;
        e->mws_bytes = 0;
    }
    if (hipMalloc((void**)&e->mws, bytes) != hipSuccess) {
        e->mws = nullptr;
        return fail(ISVD_E_NOMEM, "metrics workspace of %zu bytes", bytes);
    }
    e->mws_bytes = bytes;
    return ISVD_OK;
}

struct Exact {
    double fro2 = 0, e_inc = 0, e_opt = 0, gap = 0, ratio = 0, ortho_u = 0, ortho_v = 0;
    double angle_opt = std::nan("");
};

// out = sum of P[0:n]: thread t adds a contiguous range in order, the ranges'
// sums are added in a fixed tree order (one block of kThreads)
__global__ void __launch_bounds__(kThreads) k_sum_block(const double* __restrict__ P, int64_t n, double* out) {
    __shared__ double red[kThreads];
    const int64_t per = (n + kThreads - 1) / kThreads;
    const int64_t a = threadIdx.x * per, b = min(n, a + per);
    double s0 = 0.0, s1 = 0.0;
    int64_t i = a;
    for (; i + 1 < b; i += 2) {
        s0 += P[i];
        s1 += P[i + 1];
    }
    if (i < b) s0 += P[i];
    red[threadIdx.x] = s0 + s1;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_fill_scalars(double* d, int nd, double v, int* iv, int ni) {
    if ((int)threadIdx.x < nd) d[threadIdx.x] = v;
    if ((int)threadIdx.x < ni) iv[threadIdx.x] = 0;
}

// ||A||_F^2 and E_inc^2 (one residual pass over A), E_opt^2 = ||A||^2 minus the
// sum of the leading k squared Ritz values of a refresh computed into the
// workspace (left there for a commit; exact when its block spans all columns),
// and max |Q^T Q - I| of U and V.
// Without `ortho` (the error policy's check) the two orthogonality norms are
// left out (reported as NaN).
template <typename T>
isvd_status exact_metrics_t(isvd_engine* e, Stream& s, hipStream_t st, Exact* out, RefreshPlan* plan, bool ortho) {
    ST_TRY(refresh_compute<T>(e, s, false, st, plan));
    DevHeader h{};
    HIP_TRY(hipMemcpyAsync(&h, s.hdr, sizeof(h), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int64_t m = h.m, n = h.n;
    const int k = h.k, ld = h.ld;
    const int64_t nfro = cdiv(m, kFroRows);
    const int64_t nres = cdiv(m, 64) * cdiv(n, 64);
    const int64_t ngu = gram_parts(m), ngv = gram_parts(n);
    const int64_t gsz = (int64_t)gram_tiles(k) * 256;
    const size_t need = sizeof(double) * (size_t)(nfro + nres + (ngu + ngv) * gsz + 2 * k * k + 8);
    ST_TRY(ensure_mws(e, need));
    double* fro_p = (double*)e->mws;
    double* res_p = fro_p + nfro;
    double* gu_p = res_p + nres;
    double* gv_p = gu_p + ngu * gsz;
    double* GU = gv_p + ngv * gsz;
    double* GV = GU + k * k;
    double* scal = GV + k * k;
    const T* A = (const T*)s.A;
    const T* U = (const T*)s.U[h.cur];
    const T* V = (const T*)s.V[h.cur];
    const int64_t lda = lda_of(s.cfg);
    k_fro2_partial<T><<<(int)nfro, kThreads, 0, st>>>(A, lda, m, n, fro_p);
    k_sum_block<<<1, kThreads, 0, st>>>(fro_p, nfro, scal + 0);
    dim3 rg((unsigned)cdiv(m, 64), (unsigned)cdiv(n, 64));
    k_resid2_partial<T><<<rg, kThreads, 0, st>>>(A, lda, U, V, ld, s.S, m, n, k, res_p);
    k_sum_block<<<1, kThreads, 0, st>>>(res_p, nres, scal + 1);
    int* sw = (int*)(scal + 6);
    if (ortho) {
        k_gram_mfma<T, true><<<(int)ngu, kThreads, 0, st>>>(U, ld, m, k, gram_rpb(m), gu_p);
        k_gram_sum<<<(int)cdiv(gsz, 32), 256, 0, st>>>(gu_p, (int)ngu, k, GU);
        k_gram_mfma<T, true><<<(int)ngv, kThreads, 0, st>>>(V, ld, n, k, gram_rpb(n), gv_p);
        k_gram_sum<<<(int)cdiv(gsz, 32), 256, 0, st>>>(gv_p, (int)ngv, k, GV);
        const int nt = WideShape::NT;
        k_sym_norm2<<<1, nt, sym_norm2_lds(k), st>>>(GU, k, scal + 2, sw);
        k_sym_norm2<<<1, nt, sym_norm2_lds(k), st>>>(GV, k, scal + 3, sw + 1);
    } else {
        k_fill_scalars<<<1, 64, 0, st>>>(scal + 2, 2, std::nan(""), sw, 2);
    }
    HIP_TRY(hipGetLastError());
    std::vector<double> hs(7), sr(plan->k);
    HIP_TRY(hipMemcpyAsync(hs.data(), scal, sizeof(double) * 7, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(sr.data(), e->ws.p + plan->w.Sr, sizeof(double) * plan->k, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    out->fro2 = hs[0];
    out->e_inc = std::sqrt(std::max(hs[1], 0.0));
    // E_opt: the best approximation of the model's rank k (at most the
    // refresh's); the Gram form's Ritz values come from exact FP64 products
    // of A's entries, the A form's from products in the storage type
    double top = 0.0;
    if (!plan->gram_theta.empty()) {
        for (int q = 0; q < std::min<int>(k, (int)plan->gram_theta.size()); ++q) top += plan->gram_theta[q];
    } else {
        for (int q = 0; q < std::min(k, plan->k); ++q) top += sr[q] * sr[q];
    }
    out->e_opt = std::sqrt(std::max(hs[0] - top, 0.0));
    out->gap = out->e_inc - out->e_opt;
    out->ratio = out->e_opt > 1e-14 * std::sqrt(hs[0]) ? out->e_inc / out->e_opt : std::nan("");
    int sweeps[2];
    std::memcpy(sweeps, &hs[6], sizeof(sweeps));
    if (sweeps[0] < 0 || sweeps[1] < 0) return fail(ISVD_E_CONVERGE, "orthogonality norm did not converge");
    out->ortho_u = hs[2];
    out->ortho_v = hs[3];
    if (ortho && k > 0) {
        // theta_opt (the angle metric to the optimal subspace): the largest
        // principal angle between span(U_t) and the leading min(k, k_refresh)
        // left singular vectors of A_t, U_opt = Q_Y W from the refresh just
        // computed: M = W^T (Q_Y^T U_t), H = U_t^T U_t, theta from M and H as
        // for theta_ref (on all of U_opt's columns)
        const int b = plan->b, kq = std::min(k, plan->k);
        const int64_t chunk = 1024, nch = std::max<int64_t>(1, cdiv(m, chunk));
        const size_t need2 = sizeof(double) * (size_t)(nch * ((size_t)b * k + (size_t)k * k) + (size_t)b * k +
                                                       2 * (size_t)k * k + 16);
        ST_TRY(ensure_mws(e, need2));
        double* pp = (double*)e->mws;
        double* hp = pp + nch * b * k;
        double* Pd = hp + nch * k * k;
        double* Md = Pd + (size_t)b * k;
        double* Hd = Md + (size_t)kq * k;
        double* thd = Hd + (size_t)k * k;
        double* Rg = thd + 8;
        const T* Yq = (const T*)(e->ws.p + plan->w.Y);
        k_cross_partial<T, true><<<(int)nch, kThreads, 0, st>>>(Yq, b, b, U, ld, k, m, chunk, pp);
        k_cross_partial<T><<<(int)nch, kThreads, 0, st>>>(U, ld, k, U, ld, k, m, chunk, hp);
        k_sum_parts<double><<<(int)cdiv((int64_t)b * k, 256), 256, 0, st>>>(pp, (int)nch, (int64_t)b * k,
                                                                          (int64_t)b * k, Pd);
        k_sum_parts<double><<<(int)cdiv((int64_t)k * k, 256), 256, 0, st>>>(hp, (int)nch, (int64_t)k * k,
                                                                          (int64_t)k * k, Hd);
        k_tn_small<T><<<1, kThreads, 0, st>>>((const T*)(e->ws.p + plan->w.QU), plan->ldo, b, kq, Pd, k, Md);
        k_theta_direct<<<1, WideShape::NT, sizeof(double) * theta_lds_doubles(), st>>>(Md, Hd, k, kq, s.S, k, thd,
                                                                                       Rg);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&out->angle_opt, thd, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return ISVD_OK;
}

isvd_status exact_metrics(isvd_engine* e, Stream& s, hipStream_t st, Exact* out, RefreshPlan* plan,
                          bool ortho = true) {
    return s.esz == 8 ? exact_metrics_t<double>(e, s, st, out, plan, ortho)
                      : exact_metrics_t<float>(e, s, st, out, plan, ortho);
}

// ------------------------------------------------------------------ policies
isvd_status read_header(Stream& s, hipStream_t st, DevHeader* h) {
    HIP_TRY(hipMemcpyAsync(h, s.hdr, sizeof(DevHeader), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return ISVD_OK;
}

bool policy_needs_header(const Stream& s) {
    return s.cfg.policy.kind == ISVD_POL_ADAPTIVE || s.cfg.policy.kind == ISVD_POL_ANGLE ||
           s.cfg.policy.kind == ISVD_POL_DRIFT;
}

// Policy evaluation after the update at tick t (Algorithm 1; Section 3).
// `h` is the device header after the update when the policy needs it.
// Policy actions of one tick that its caller runs together.
struct Deferred {
    std::vector<Stream*> refresh;   // fired refreshes
    std::vector<Stream*> shrink;    // adaptive-rank shrinks
    std::vector<Stream*> checks;    // error-policy checks due (batched)
};
bool seg_eligible(const Stream& s);

// With `defer`, a refresh that the policy fires, or an adaptive shrink, is
// appended to it (the caller runs the tick's actions together) instead of
// running here.
constexpr int64_t kBf16AngleCheck = 32;   // BF16-rotation streams: updates between direct angle measurements
isvd_status after_update(isvd_engine* e, Stream& s, hipStream_t st, const DevHeader* h,
                         Deferred* defer = nullptr) {
    const isvd_policy& p = s.cfg.policy;
    auto refresh = [&]() -> isvd_status {
        if (defer) {
            defer->refresh.push_back(&s);
            return ISVD_OK;
        }
        return do_refresh(e, s, false, true, st);
    };
    if (p.kind == ISVD_POL_PERIODIC) {
        if (p.period > 0 && s.t % p.period == 0) return refresh();
        return ISVD_OK;
    }
    if (p.kind == ISVD_POL_ERROR) {
        if (p.check_every <= 0 || s.t % p.check_every != 0 || s.t - s.t_last < p.t_min) return ISVD_OK;
        if (defer && e->seg_refresh && seg_eligible(s)) {
            defer->checks.push_back(&s);
            return ISVD_OK;
        }
        Exact ex;
        RefreshPlan plan;
        ST_TRY(exact_metrics(e, s, st, &ex, &plan, false));
        s.last_ratio = ex.ratio;
        if (ex.ratio > p.gamma) return do_refresh(e, s, false, true, st, &plan);
        return ISVD_OK;
    }
    if (p.kind == ISVD_POL_DRIFT) {
        // the step angle of U of the update just applied, from the header
        DevHeader hh;
        if (!h) {
            ST_TRY(read_header(s, st, &hh));
            h = &hh;
        }
        if (std::isfinite(h->step_angle_u)) s.drift_acc += h->step_angle_u;
        if (s.t - s.t_last >= std::max<int64_t>(p.t_min, 1) && s.drift_acc > p.theta_max) return refresh();
        return ISVD_OK;
    }
    if (p.kind == ISVD_POL_ANGLE) {
        if (s.t - s.t_last < std::max<int64_t>(p.t_min, 1)) return ISVD_OK;
        if (s.bf16 && s.t % kBf16AngleCheck == 0) {
            // The trackers follow the core's exact rotations, not the BF16
            // rounding the stored bases take on: every kBf16AngleCheck updates
            // the angle is measured from the stored U (and M, H restart from it)
            double theta = 0.0;
            ST_TRY(direct_trackers(e, s, st, &theta, s.TM, s.TH, s.kc));
            if (theta > p.theta_max) return refresh();
            return ISVD_OK;
        }
        DevHeader hh;
        if (!h) {
            ST_TRY(read_header(s, st, &hh));
            h = &hh;
        }
        if (h->angle_ref > p.theta_max) return refresh();
        return ISVD_OK;
    }
    if (p.kind == ISVD_POL_ADAPTIVE) {
        DevHeader hh;
        if (!h) {
            ST_TRY(read_header(s, st, &hh));
            h = &hh;
        }
        // the device decides how many triplets an append keeps; follow it
        if (h->k > s.k_target) s.grow_pending = false;
        s.k_target = h->k;
        const int kmax = p.k_max > 0 ? p.k_max : s.cfg.k;
        const int kmin = std::max(1, p.k_min);
        const double s2 = h->sigma2, N = h->N;
        const bool low = N > 0.0 && s2 / N < p.tau - p.band;
        const bool novel = (h->last_kind == kRow || h->last_kind == kCol) && h->novelty > p.eta;
        if (low || novel) {
            if (s.k_target < kmax) s.grow_pending = true;
        } else if (h->k > kmin && N > 0.0 && (s2 - h->sigma_last * h->sigma_last) / N >= p.tau + p.band) {
            if (defer) {
                defer->shrink.push_back(&s);
            } else {
                k_shrink<<<1, 1, 0, st>>>(s.hdr, s.S);
                HIP_TRY(hipGetLastError());
            }
            s.k_target = h->k - 1;
            s.grow_pending = false;
        }
        if (p.period > 0 && s.t % p.period == 0) return refresh();
        return ISVD_OK;
    }
    return ISVD_OK;
}

// The refreshes fired by one tick's policies, concurrently: refresh i runs on
// lane i mod kRefreshLanes with the lane's workspace, after everything the
// caller's stream holds so far (the tick and its policy actions); the caller's
// stream then waits for the lanes.  The streams of `list` are distinct.
constexpr int kRefreshLanes = 8;
isvd_status ensure_refresh_lanes(isvd_engine* e) {
    if (!e->rlanes.empty()) return ISVD_OK;
    e->rlanes.resize(kRefreshLanes);
    for (auto& l : e->rlanes) {
        HIP_TRY(hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&l.ev, hipEventDisableTiming));
        l.ws.defer_free = true;
        l.jobs.defer_free = true;
    }
    e->seg_cws.defer_free = true;
    e->seg_cjobs.defer_free = true;
    for (auto& q : e->seg_slot) HIP_TRY(hipEventCreateWithFlags(&q.ev, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&e->ev_policies, hipEventDisableTiming));
    HIP_TRY(hipMalloc((void**)&e->dsweeps, sizeof(int) * kMaxLiveStreams));
    HIP_TRY(hipHostMalloc((void**)&e->rsweeps, sizeof(int) * kMaxLiveStreams, hipHostMallocDefault));
    return ISVD_OK;
}

// The initial TruncatedSVD of a new stream on the next refresh lane, after
// everything `st` holds (the copy of A_0 and its norm); the stream is busy
// until it is done.
isvd_status init_on_lane(isvd_engine* e, Stream& s, hipStream_t st) {
    ST_TRY(ensure_refresh_lanes(e));
    auto& lane = e->rlanes[e->next_lane];
    e->next_lane = (e->next_lane + 1) % kRefreshLanes;
    if (!lane.ws.retired.empty() && hipStreamQuery(lane.st) == hipSuccess) free_retired(lane.ws);
    HIP_TRY(hipEventRecord(e->ev_policies, st));
    HIP_TRY(hipStreamWaitEvent(lane.st, e->ev_policies, 0));
    ST_TRY(do_refresh(e, s, true, true, lane.st, nullptr, nullptr, e->dsweeps + s.slot, &lane.ws));
    HIP_TRY(hipMemcpyAsync(e->rsweeps + s.slot, e->dsweeps + s.slot, sizeof(int), hipMemcpyDeviceToHost, lane.st));
    HIP_TRY(hipEventRecord(s.ev_ready, lane.st));
    s.refreshing = true;
    HIP_TRY(hipEventRecord(lane.ev, lane.st));
    lane.pending = true;
    return ISVD_OK;
}

// ------------------------------------------------- segmented refresh batches
// The tick-fired A-form refreshes of FP32 streams, phase by phase: each
// phase is one launch over every stream of the batch (split by the block
// width NB where the kernel is specialised on it), with each stream's
// workspace in its own region of one buffer.  The per-stream steps are those
// of refresh_compute and refresh_commit (with the reference stored), so the
// results are bitwise theirs.
enum SegKind { kSegStart, kSegGram, kSegGramSum, kSegChol, kSegNN, kSegTN, kSegTnSum, kSegSmall, kSegRot,
               kSegRotTiled, kSegSvd, kSegCommit };

struct SegProgram {
    struct L {
        int kind, variant, njobs, blocks;
        size_t jobs, begin;
    };
    std::vector<char> host;
    std::vector<L> launches;
    size_t put(const void* p, size_t bytes) {
        const size_t o = align_up(host.size(), 16);
        host.resize(o + bytes);
        std::memcpy(host.data() + o, p, bytes);
        return o;
    }
    template <class J>
    void add(int kind, int variant, const std::vector<J>& jobs, const std::vector<int>& blocks) {
        if (jobs.empty()) return;
        std::vector<int> begin(jobs.size() + 1, 0);
        for (size_t q = 0; q < jobs.size(); ++q) begin[q + 1] = begin[q] + blocks[q];
        L l{kind, variant, (int)jobs.size(), begin.back(), 0, 0};
        l.jobs = put(jobs.data(), sizeof(J) * jobs.size());
        l.begin = put(begin.data(), sizeof(int) * begin.size());
        launches.push_back(l);
    }
};

struct SegRef {
    Stream* s;
    int k, b, ldo, cur, kw, iters;
    bool exact;
    int64_t m, n, lda;
    int ld;
    WsLayout w;
    size_t off;
    char* ws = nullptr;
};

// CholQR passes on the block `Y(r)` (rows(r) x b) of every ref, as cholqr()
void seg_cholqr(SegProgram& P, std::vector<SegRef>& g, const std::function<float*(SegRef&)>& Y,
                const std::function<int64_t(SegRef&)>& rows, int passes, bool want_R) {
    for (int pass = 0; pass < passes; ++pass) {
        std::vector<SjGram> gj;
        std::vector<SjGramSum> sj;
        std::vector<SjChol> cj;
        std::vector<SjSmallGemm> mj;
        std::vector<SjRot> rj;
        std::vector<int> gb, sb, ones, rb, mb;
        std::vector<SjNN> nj[9];
        std::vector<int> nbk[9];
        for (SegRef& r : g) {
            const int64_t rw = rows(r);
            char* ws = r.ws;
            float* y = Y(r);
            const int nparts = (int)gram_parts(rw);
            gj.push_back(SjGram{y, (double*)(ws + r.w.Gp), rw, gram_rpb(rw), r.b, r.b});
            gb.push_back(nparts);
            sj.push_back(SjGramSum{(const double*)(ws + r.w.Gp), (double*)(ws + r.w.G), nparts, r.b});
            sb.push_back((int)cdiv(gram_tiles(r.b) * 256, 32));
            cj.push_back(SjChol{(const double*)(ws + r.w.G), (double*)(ws + (want_R && pass == 0 ? r.w.Racc : r.w.R)),
                                (float*)(ws + r.w.RinvT), (int*)(ws + r.w.flag), r.b});
            ones.push_back(1);
            if (r.b % 4 == 0) {
                const int nb = std::min(8, (r.b + 15) / 16);
                nj[nb].push_back(SjNN{y, (const float*)(ws + r.w.RinvT), y, r.b, rw, r.b, r.b, r.b});
                nbk[nb].push_back((int)cdiv(rw, 128));
            } else {
                rj.push_back(SjRot{y, y, (const float*)(ws + r.w.RinvT), nullptr, rw, r.b, r.b, r.b});
                rb.push_back((int)cdiv(rw, 16));
            }
            if (want_R && pass == 1) {
                mj.push_back(SjSmallGemm{(const double*)(ws + r.w.R), (const double*)(ws + r.w.Racc),
                                         (double*)(ws + r.w.Rtmp), r.b});
                mb.push_back((int)cdiv(r.b * r.b, 256));
            }
        }
        P.add(kSegGram, 0, gj, gb);
        P.add(kSegGramSum, 0, sj, sb);
        P.add(kSegChol, 0, cj, ones);
        for (int nb = 1; nb <= 8; ++nb) P.add(kSegNN, nb, nj[nb], nbk[nb]);
        P.add(kSegRot, 0, rj, rb);
        P.add(kSegSmall, 0, mj, mb);
    }
}

// A X -> Y for every ref (rows m, inner n)
void seg_ax(SegProgram& P, std::vector<SegRef>& g) {
    std::vector<SjNN> nj[9];
    std::vector<int> nbk[9];
    for (SegRef& r : g) {
        const int nb = std::min(8, (r.b + 15) / 16);
        nj[nb].push_back(SjNN{(const float*)r.s->A, (const float*)(r.ws + r.w.X), (float*)(r.ws + r.w.Y), r.lda, r.m,
                              r.n, r.b, r.b});
        nbk[nb].push_back((int)cdiv(r.m, 128));
    }
    for (int nb = 1; nb <= 8; ++nb) P.add(kSegNN, nb, nj[nb], nbk[nb]);
}

// One group of refs sharing (exact, iters): the launches of refresh_compute<float>
// in the A form (the Rayleigh-Ritz sweep counts into e->dsweeps).
void seg_compute(isvd_engine* e, SegProgram& P, std::vector<SegRef>& g) {
    if (g.empty()) return;
    const bool exact = g[0].exact;
    const int iters = g[0].iters;
    auto X = [](SegRef& r) { return (float*)(r.ws + r.w.X); };
    auto Y = [](SegRef& r) { return (float*)(r.ws + r.w.Y); };
    auto nrows = [](SegRef& r) { return r.n; };
    auto mrows = [](SegRef& r) { return r.m; };
    {
        std::vector<SjStart> j;
        std::vector<int> bl;
        for (SegRef& r : g) {
            j.push_back(SjStart{X(r), (const float*)r.s->V[r.cur], (int*)(r.ws + r.w.flag), r.n,
                                0x5eedull + (uint64_t)r.s->t, r.b, r.b, r.ld, r.kw, exact ? 1 : 0});
            bl.push_back((int)cdiv(r.n * r.b, 256));
        }
        P.add(kSegStart, 0, j, bl);
    }
    if (!exact) seg_cholqr(P, g, X, nrows, iters > 0 ? 1 : 2, false);
    for (int it = 0; it < iters; ++it) {
        seg_ax(P, g);
        seg_cholqr(P, g, Y, mrows, 1, false);
        std::vector<SjTN> tj[9];
        std::vector<int> tb[9];
        std::vector<SjTnSum> sj;
        std::vector<int> sb;
        for (SegRef& r : g) {
            const int64_t ncb = cdiv(r.n, kTnCols), nch = tn_chunks(r.m, r.n), per = ncb * kTnDump;
            const int nb = std::min(8, (r.b + 15) / 16);
            tj[nb].push_back(SjTN{(const float*)r.s->A, Y(r), (float*)(r.ws + r.w.Zp), r.lda, r.m, r.n,
                                  cdiv(r.m, nch), r.b, (int)ncb});
            tb[nb].push_back((int)(ncb * nch));
            sj.push_back(SjTnSum{(const float*)(r.ws + r.w.Zp), X(r), per, r.n, (int)nch, r.b, r.b});
            sb.push_back((int)cdiv(per, 256));
        }
        for (int nb = 1; nb <= 8; ++nb) P.add(kSegTN, nb, tj[nb], tb[nb]);
        P.add(kSegTnSum, 0, sj, sb);
        seg_cholqr(P, g, X, nrows, it + 1 == iters ? 2 : 1, false);
    }
    seg_ax(P, g);
    seg_cholqr(P, g, Y, mrows, 2, true);
    {
        std::vector<SjSvd> j;
        std::vector<int> ones;
        for (SegRef& r : g) {
            j.push_back(SjSvd{(const double*)(r.ws + r.w.Rtmp), (double*)(r.ws + r.w.Sr), (float*)(r.ws + r.w.QU),
                              (float*)(r.ws + r.w.QV), e->dsweeps + r.s->slot, r.b, r.k, r.ldo});
            ones.push_back(1);
        }
        P.add(kSegSvd, 0, j, ones);
    }
}

// The launches of refresh_commit<float> with the reference stored, for refs
// whose refresh seg_compute has left in their workspace regions.
void seg_commit(SegProgram& P, std::vector<SegRef>& g) {
    auto X = [](SegRef& r) { return (float*)(r.ws + r.w.X); };
    auto Y = [](SegRef& r) { return (float*)(r.ws + r.w.Y); };
    {
        std::vector<SjRot> j;
        std::vector<int> bl;
        for (SegRef& r : g) {
            const int nxt = r.cur ^ 1;
            j.push_back(SjRot{Y(r), (float*)r.s->U[nxt], (const float*)(r.ws + r.w.QU), (float*)r.s->Uref, r.m, r.b,
                              r.ldo, r.b});
            bl.push_back((int)cdiv(r.m, 16));
            j.push_back(SjRot{X(r), (float*)r.s->V[nxt], (const float*)(r.ws + r.w.QV), nullptr, r.n, r.b, r.ldo,
                              r.b});
            bl.push_back((int)cdiv(r.n, 16));
        }
        P.add(kSegRotTiled, 0, j, bl);
    }
    {
        std::vector<SjCommit> j;
        std::vector<int> ones;
        for (SegRef& r : g) {
            Stream& s = *r.s;
            SjCommit c{};
            c.hdr = s.hdr;
            c.S_out = s.S;
            c.S = (const double*)(r.ws + r.w.Sr);
            if (s.wbuf) {
                const size_t w = (size_t)s.kc * s.kc;
                c.W[0] = s.wbuf;
                c.W[1] = s.wbuf + w;
                c.W[2] = s.wbuf + 2 * w;
                c.W[3] = s.wbuf + 3 * w;
            }
            c.TM = s.TM;
            c.TH = s.TH;
            c.k = r.k;
            c.ld = r.ldo;
            c.kcw = s.kc;
            c.kct = s.kc;
            j.push_back(c);
            ones.push_back(1);
        }
        P.add(kSegCommit, 0, j, ones);
    }
}

isvd_status seg_launch(const SegProgram::L& l, char* dev, hipStream_t st) {
    const void* jobs = dev + l.jobs;
    const int* begin = (const int*)(dev + l.begin);
    const int n = l.njobs, B = l.blocks;
    switch (l.kind) {
        case kSegStart: k_seg_start<<<B, 256, 0, st>>>((const SjStart*)jobs, begin, n); break;
        case kSegGram: k_seg_gram<<<B, kThreads, 0, st>>>((const SjGram*)jobs, begin, n); break;
        case kSegGramSum: k_seg_gram_sum<<<B, 256, 0, st>>>((const SjGramSum*)jobs, begin, n); break;
        case kSegChol: k_seg_chol<<<n, kCholThreads, 0, st>>>((const SjChol*)jobs); break;
        case kSegNN:
            switch (l.variant) {
#define ISVD_SNN(NB) case NB: k_seg_nn<NB><<<B, kThreads, 0, st>>>((const SjNN*)jobs, begin, n); break;
                ISVD_SNN(1) ISVD_SNN(2) ISVD_SNN(3) ISVD_SNN(4) ISVD_SNN(5) ISVD_SNN(6) ISVD_SNN(7) ISVD_SNN(8)
#undef ISVD_SNN
                default: return fail(ISVD_E_INVAL, "segmented product width %d", l.variant);
            }
            break;
        case kSegTN:
            switch (l.variant) {
#define ISVD_STN(NB) case NB: k_seg_tn<NB><<<B, kThreads, 0, st>>>((const SjTN*)jobs, begin, n); break;
                ISVD_STN(1) ISVD_STN(2) ISVD_STN(3) ISVD_STN(4) ISVD_STN(5) ISVD_STN(6) ISVD_STN(7) ISVD_STN(8)
#undef ISVD_STN
                default: return fail(ISVD_E_INVAL, "segmented product width %d", l.variant);
            }
            break;
        case kSegTnSum: k_seg_tn_sum<<<B, 256, 0, st>>>((const SjTnSum*)jobs, begin, n); break;
        case kSegSmall: k_seg_small_gemm<<<B, 256, 0, st>>>((const SjSmallGemm*)jobs, begin, n); break;
        case kSegRot: k_seg_rot<false><<<B, kThreads, 0, st>>>((const SjRot*)jobs, begin, n); break;
        case kSegRotTiled: k_seg_rot<true><<<B, kThreads, 0, st>>>((const SjRot*)jobs, begin, n); break;
        case kSegSvd:
            k_seg_svd<<<n, RRShape::NT, sizeof(double) * svd_noj_lds_doubles(), st>>>((const SjSvd*)jobs);
            break;
        case kSegCommit: k_seg_commit<<<n, 256, 0, st>>>((const SjCommit*)jobs); break;
        default: return fail(ISVD_E_INVAL, "segmented launch kind %d", l.kind);
    }
    HIP_TRY(hipGetLastError());
    return ISVD_OK;
}

// Can stream s take the segmented batch?  FP32 storage (BF16 rotations
// included: the refresh works on A) and the A form.
bool seg_eligible(const Stream& s) {
    if (s.esz != 4) return false;
    int k = 0, b = 0;
    refresh_block(s, &k, &b);
    return k >= 1 && b >= k && !gram_form(s, b);
}

// The refresh of stream s as a batch entry, its header from e->hdr_mirror;
// its workspace region starts at *total, which moves past it.
SegRef seg_ref(isvd_engine* e, Stream& s, size_t* total, bool init = false) {
    DevHeader h{};
    if (init) {
        h.ld = 4;   // the start block takes no column of V
    } else {
        h = e->hdr_mirror[s.slot];
    }
    SegRef r{};
    r.s = &s;
    refresh_block(s, &r.k, &r.b);
    r.m = s.m;
    r.n = s.n;
    r.lda = lda_of(s.cfg);
    r.exact = r.b == r.n;
    r.iters = r.exact ? 0 : s.cfg.refresh_iters >= 0 ? s.cfg.refresh_iters : (init ? 8 : 3);
    r.ldo = round4(r.k);
    r.cur = h.cur;
    r.ld = h.ld;
    r.kw = std::min(h.k, r.b);
    r.w = ws_layout(r.m, r.n, r.b, 4);
    r.off = *total;
    *total = align_up(*total + r.w.total, 256);
    return r;
}

// The job tables of P to the device buffer `dev` (grown as needed), through
// the next pinned staging slot, on stream q.
isvd_status seg_upload(isvd_engine* e, const SegProgram& P, WsBuf& dev, hipStream_t q) {
    const size_t bytes = std::max<size_t>(P.host.size(), 16);
    auto& slot = e->seg_slot[e->seg_next];
    e->seg_next = (e->seg_next + 1) % 4;
    if (slot.used) HIP_TRY(hipEventSynchronize(slot.ev));
    if (slot.bytes < bytes) {
        if (slot.host) HIP_TRY(hipHostFree(slot.host));
        slot.host = nullptr;
        slot.bytes = 0;
        const size_t want = bytes + bytes / 2;
        HIP_TRY(hipHostMalloc((void**)&slot.host, want, hipHostMallocDefault));
        slot.bytes = want;
    }
    std::memcpy(slot.host, P.host.data(), P.host.size());
    ST_TRY(ensure_ws(dev, bytes));
    HIP_TRY(hipMemcpyAsync(dev.p, slot.host, P.host.size(), hipMemcpyHostToDevice, q));
    HIP_TRY(hipEventRecord(slot.ev, q));
    slot.used = true;
    return ISVD_OK;
}

// Host state after a committed refresh, as do_refresh / refresh_commit /
// defer_after_refresh leave it (a stream's initial SVD counts no refresh).
void seg_host_commit(Stream& s, const SegRef& r, bool init = false) {
    s.refresh_rounds = 0;
    s.refresh_converged = true;
    s.k_target = r.k;
    if (s.wbuf) {
        s.defer_pending = 0;
        s.defer_period = defer_period_for(s);
    }
    s.have_refresh_time = true;
    if (!init) {
        s.n_refresh += 1;
        s.t_last = s.t;
    }
    s.drift_acc = 0.0;
}

// The refreshes of `list` (all seg_eligible, distinct, their headers in
// e->hdr_mirror) as one segmented batch on refresh lane `L` (its workspace
// holds the streams' regions), after what the lane holds; with `init`, the
// initial TruncatedSVDs of new streams (random start block).
isvd_status refresh_segmented(isvd_engine* e, const std::vector<Stream*>& list, isvd_engine::RefreshLane& L,
                              bool init = false) {
    hipStream_t lane = L.st;
    std::vector<SegRef> refs;
    size_t total = 0;
    for (Stream* sp : list) refs.push_back(seg_ref(e, *sp, &total, init));
    if (hipStreamQuery(lane) == hipSuccess) {
        free_retired(L.ws);
        free_retired(L.jobs);
    }
    ST_TRY(ensure_ws(L.ws, std::max<size_t>(total, 256)));
    for (SegRef& r : refs) r.ws = L.ws.p + r.off;
    // groups of equal (exact, iters): the same launch sequence
    std::map<std::pair<int, int>, std::vector<SegRef>> groups;
    for (SegRef& r : refs) groups[{r.exact ? 1 : 0, r.iters}].push_back(r);
    SegProgram P;
    for (auto& kv : groups) {
        seg_compute(e, P, kv.second);
        seg_commit(P, kv.second);
    }
    ST_TRY(seg_upload(e, P, L.jobs, lane));
    for (Stream* sp : list) HIP_TRY(hipEventRecord(sp->ev_r0, lane));
    for (const auto& l : P.launches) ST_TRY(seg_launch(l, L.jobs.p, lane));
    for (SegRef& r : refs) {
        Stream& s = *r.s;
        seg_host_commit(s, r, init);
        HIP_TRY(hipEventRecord(s.ev_r1, lane));
        HIP_TRY(hipMemcpyAsync(e->rsweeps + s.slot, e->dsweeps + s.slot, sizeof(int), hipMemcpyDeviceToHost, lane));
        HIP_TRY(hipEventRecord(s.ev_ready, lane));
        s.refreshing = true;
    }
    return ISVD_OK;
}

// Error-policy checks of one tick, batched (Sec. 3.2, eq. error-refresh-rule):
// for the FP32 streams whose refresh runs in the A form, the TruncatedSVD of
// every check is computed in one segmented batch on the caller's stream, the
// residual and norm passes follow per stream, one copy and one wait bring
// every stream's E_inc, ||A||^2 and Ritz values back, and the streams whose
// ratio exceeds gamma commit their computed refresh in one more segmented
// batch.  Each step is exact_metrics' and do_refresh's own, so decisions and
// states are bitwise those of the checks run one by one.
isvd_status check_batch(isvd_engine* e, const std::vector<Stream*>& list, hipStream_t st) {
    ST_TRY(ensure_refresh_lanes(e));
    HIP_TRY(hipMemcpyAsync(e->hdr_mirror, e->hdr_dev, sizeof(DevHeader) * e->hdr_hi, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (!e->seg_cws.retired.empty()) free_retired(e->seg_cws);
    if (!e->seg_cjobs.retired.empty()) free_retired(e->seg_cjobs);
    std::vector<SegRef> refs;
    std::vector<size_t> mo;       // per ref: offset of its metric partials in its region
    size_t total = 0;
    for (Stream* sp : list) {
        SegRef r = seg_ref(e, *sp, &total);
        const int64_t nres = cdiv(r.m, 64) * cdiv(r.n, 64);
        mo.push_back(total);
        total = align_up(total + sizeof(double) * (size_t)(nres + 8), 256);
        refs.push_back(r);
    }
    ST_TRY(ensure_ws(e->seg_cws, std::max<size_t>(total, 256)));
    for (SegRef& r : refs) r.ws = e->seg_cws.p + r.off;
    std::map<std::pair<int, int>, std::vector<SegRef>> groups;
    for (SegRef& r : refs) groups[{r.exact ? 1 : 0, r.iters}].push_back(r);
    SegProgram P;
    for (auto& kv : groups) seg_compute(e, P, kv.second);
    ST_TRY(seg_upload(e, P, e->seg_cjobs, st));
    for (const auto& l : P.launches) ST_TRY(seg_launch(l, e->seg_cjobs.p, st));
    // E_inc^2 and ||A||^2 per stream (as exact_metrics), then one copy back
    const size_t per = 8 + 2 * kMaxBlock;   // doubles per stream in the host buffer
    if (e->chk_host_n < refs.size() * per) {
        if (e->chk_host) HIP_TRY(hipHostFree(e->chk_host));
        e->chk_host = nullptr;
        e->chk_host_n = 0;
        HIP_TRY(hipHostMalloc((void**)&e->chk_host, sizeof(double) * refs.size() * per * 2, hipHostMallocDefault));
        e->chk_host_n = refs.size() * per * 2;
    }
    for (size_t q = 0; q < refs.size(); ++q) {
        SegRef& r = refs[q];
        Stream& s = *r.s;
        const DevHeader& h = e->hdr_mirror[s.slot];
        double* fro_p = (double*)(r.ws + r.w.fro);
        double* res_p = (double*)(e->seg_cws.p + mo[q]);
        const int64_t nres = cdiv(r.m, 64) * cdiv(r.n, 64);
        double* scal = res_p + nres;
        const float* A = (const float*)s.A;
        const int64_t nfro = cdiv(r.m, kFroRows);
        k_fro2_partial<float><<<(int)nfro, kThreads, 0, st>>>(A, r.lda, r.m, r.n, fro_p);
        k_sum_block<<<1, kThreads, 0, st>>>(fro_p, nfro, scal + 0);
        dim3 rg((unsigned)cdiv(r.m, 64), (unsigned)cdiv(r.n, 64));
        k_resid2_partial<float><<<rg, kThreads, 0, st>>>(A, r.lda, (const float*)s.U[h.cur], (const float*)s.V[h.cur],
                                                        h.ld, s.S, r.m, r.n, h.k, res_p);
        k_sum_block<<<1, kThreads, 0, st>>>(res_p, nres, scal + 1);
        HIP_TRY(hipGetLastError());
        double* hb = e->chk_host + q * per;
        HIP_TRY(hipMemcpyAsync(hb, scal, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hb + 2, e->dsweeps + s.slot, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hb + 8, r.ws + r.w.Sr, sizeof(double) * r.k, hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<SegRef> fire;
    for (size_t q = 0; q < refs.size(); ++q) {
        SegRef& r = refs[q];
        Stream& s = *r.s;
        const DevHeader& h = e->hdr_mirror[s.slot];
        const double* hb = e->chk_host + q * per;
        const double fro2 = hb[0];
        const double e_inc = std::sqrt(std::max(hb[1], 0.0));
        double top = 0.0;
        for (int j = 0; j < std::min(h.k, r.k); ++j) top += hb[8 + j] * hb[8 + j];
        const double e_opt = std::sqrt(std::max(fro2 - top, 0.0));
        const double ratio = e_opt > 1e-14 * std::sqrt(fro2) ? e_inc / e_opt : std::nan("");
        s.last_ratio = ratio;
        if (ratio > s.cfg.policy.gamma) {
            int sweeps = 0;
            std::memcpy(&sweeps, hb + 2, sizeof(int));
            if (sweeps < 0) return fail(ISVD_E_CONVERGE, "Rayleigh-Ritz Jacobi did not converge");
            fire.push_back(r);
        }
    }
    if (fire.empty()) return ISVD_OK;
    SegProgram C;
    seg_commit(C, fire);
    ST_TRY(seg_upload(e, C, e->seg_cjobs, st));
    for (SegRef& r : fire) HIP_TRY(hipEventRecord(r.s->ev_r0, st));
    for (const auto& l : C.launches) ST_TRY(seg_launch(l, e->seg_cjobs.p, st));
    for (SegRef& r : fire) {
        seg_host_commit(*r.s, r);
        HIP_TRY(hipEventRecord(r.s->ev_r1, st));
    }
    return ISVD_OK;
}

isvd_status refresh_batch(isvd_engine* e, const std::vector<Stream*>& all, hipStream_t st) {
    ST_TRY(ensure_refresh_lanes(e));
    // FP32 streams refreshing in the A form go as one segmented batch (when
    // there are at least two of them) on the next refresh lane in turn, so
    // the batches of successive ticks overlap; the rest one by one on the lanes
    std::vector<Stream*> seg, list;
    for (Stream* sp : all) (e->seg_refresh && seg_eligible(*sp) ? seg : list).push_back(sp);
    if (seg.size() < 2) {
        list = all;
        seg.clear();
    }
    const int cnt = (int)list.size();
    // buffers retired by workspace growth go once their lane has drained
    for (auto& l : e->rlanes)
        if (!l.ws.retired.empty() && hipStreamQuery(l.st) == hipSuccess) free_retired(l.ws);
    // headers after every policy action of the tick (one copy, one wait)
    HIP_TRY(hipMemcpyAsync(e->hdr_mirror, e->hdr_dev, sizeof(DevHeader) * e->hdr_hi, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipEventRecord(e->ev_policies, st));
    if (!seg.empty()) {
        auto& lane = e->rlanes[e->seg_lane];
        e->seg_lane = (e->seg_lane + 1) % kRefreshLanes;
        HIP_TRY(hipStreamWaitEvent(lane.st, e->ev_policies, 0));
        ST_TRY(refresh_segmented(e, seg, lane));
        HIP_TRY(hipEventRecord(lane.ev, lane.st));
        lane.pending = true;
    }
    if (cnt == 0) return ISVD_OK;
    const int used = std::min(cnt, kRefreshLanes);
    for (int l = 0; l < used; ++l) HIP_TRY(hipStreamWaitEvent(e->rlanes[l].st, e->ev_policies, 0));
    // each lane's refreshes are queued by a host thread of its own (the
    // launches of one refresh cost about as much host time as the device
    // spends on a small stream); the streams are distinct, so the threads
    // share no mutable state.  Nothing waits for the lanes here: a stream
    // under refresh is marked, and later work on it waits for its ev_ready.
    std::vector<isvd_status> rcs(used, ISVD_OK);
    std::vector<std::string> msgs(used);
    auto run_lane = [&](int l) {
        (void)hipSetDevice(e->device);
        auto& lane = e->rlanes[l];
        for (int i = l; i < cnt && rcs[l] == ISVD_OK; i += kRefreshLanes) {
            Stream& s = *list[i];
            isvd_status rc = do_refresh(e, s, false, true, lane.st, nullptr, e->hdr_mirror + s.slot,
                                        e->dsweeps + s.slot, &lane.ws);
            if (rc == ISVD_OK &&
                (hipMemcpyAsync(e->rsweeps + s.slot, e->dsweeps + s.slot, sizeof(int), hipMemcpyDeviceToHost,
                                lane.st) != hipSuccess ||
                 hipEventRecord(s.ev_ready, lane.st) != hipSuccess))
                rc = fail(ISVD_E_DEVICE, "refresh lane bookkeeping failed");
            if (rc == ISVD_OK) s.refreshing = true;
            rcs[l] = rc;
        }
        if (rcs[l] != ISVD_OK) msgs[l] = isvd_last_error();
    };
    std::vector<std::thread> workers;
    for (int l = 1; l < used; ++l) workers.emplace_back(run_lane, l);
    run_lane(0);
    for (auto& t : workers) t.join();
    for (int l = 0; l < used; ++l) {
        HIP_TRY(hipEventRecord(e->rlanes[l].ev, e->rlanes[l].st));
        e->rlanes[l].pending = true;
    }
    for (int l = 0; l < used; ++l)
        if (rcs[l] != ISVD_OK) return fail(rcs[l], "%s", msgs[l].c_str());
    return ISVD_OK;
}

// A stream whose lane refresh has finished: check its Rayleigh-Ritz sweep count.
isvd_status settle(isvd_engine* e, Stream& s, bool wait) {
    if (!s.refreshing) return ISVD_OK;
    if (wait) {
        HIP_TRY(hipEventSynchronize(s.ev_ready));
    } else if (hipEventQuery(s.ev_ready) != hipSuccess) {
        return ISVD_OK;
    }
    s.refreshing = false;
    if (e->rsweeps[s.slot] < 0) return fail(ISVD_E_CONVERGE, "Rayleigh-Ritz Jacobi did not converge");
    return ISVD_OK;
}

// Work queued on `st` after this waits for every refresh lane.
isvd_status join_refreshes(isvd_engine* e, hipStream_t st) {
    for (auto& l : e->rlanes)
        if (l.pending) {
            HIP_TRY(hipStreamWaitEvent(st, l.ev, 0));
            l.pending = false;
        }
    return ISVD_OK;
}

isvd_status stage_payload(Stream& s, const void* src, int64_t len, int32_t dtype, int32_t on_device,
                          hipStream_t st, const void** out) {
    const bool want64 = s.esz == 8;
    const bool is64 = dtype == ISVD_DTYPE_F64;
    if (dtype != ISVD_DTYPE_F32 && dtype != ISVD_DTYPE_F64) return fail(ISVD_E_INVAL, "bad dtype %d", dtype);
    if (!src) return fail(ISVD_E_INVAL, "null payload");
    if (on_device) {
        if (want64 == is64) {
            *out = src;
            return ISVD_OK;
        }
        if (is64)
            k_copy2d<double, float><<<(int)cdiv(len, 256), 256, 0, st>>>((const double*)src, len, (float*)s.stage, len, 1, len);
        else
            k_copy2d<float, double><<<(int)cdiv(len, 256), 256, 0, st>>>((const float*)src, len, (double*)s.stage, len, 1, len);
        HIP_TRY(hipGetLastError());
    } else {
        for (int64_t q = 0; q < len; ++q) {
            double v = is64 ? ((const double*)src)[q] : (double)((const float*)src)[q];
            if (!std::isfinite(v)) return fail(ISVD_E_NONFINITE, "payload entry %lld is not finite", (long long)q);
        }
        if (want64 == is64) {
            HIP_TRY(hipMemcpyAsync(s.stage, src, (size_t)s.esz * len, hipMemcpyHostToDevice, st));
            HIP_TRY(hipStreamSynchronize(st));
        } else {
            std::vector<char> tmp((size_t)s.esz * len);
            if (want64)
                for (int64_t q = 0; q < len; ++q) ((double*)tmp.data())[q] = ((const float*)src)[q];
            else
                for (int64_t q = 0; q < len; ++q) ((float*)tmp.data())[q] = (float)((const double*)src)[q];
            HIP_TRY(hipMemcpyAsync(s.stage, tmp.data(), tmp.size(), hipMemcpyHostToDevice, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
    }
    *out = s.stage;
    return ISVD_OK;
}

// Triplets an append keeps: one more than the rank while adaptive growth is
// pending (the rank grows only if the append brings a new direction).
int k_keep_for(const Stream& s, int kind) {
    const isvd_policy& p = s.cfg.policy;
    if (p.kind == ISVD_POL_ADAPTIVE && s.grow_pending && kind != kEntry) {
        const int kmax = p.k_max > 0 ? p.k_max : s.cfg.k;
        if (s.k_target < kmax) return s.k_target + 1;
    }
    return s.k_target;
}

isvd_status single_update(isvd_engine* e, Stream& s, int kind, const void* payload, int64_t i, int64_t j,
                          double delta, hipStream_t st) {
    std::vector<Group> groups(1);
    Group& g = groups[0];
    g.fp64 = s.esz == 8;
    g.bf16 = s.bf16;
    g.kc = s.kc;
    g.rows = rows_for(e, g.kc, g.fp64);
    g.var = var_for(e, g.kc, g.fp64);
    Req r = make_req(e, s, kind, payload, i, j, delta, k_keep_for(s, kind));
    g.all.push_back(r);
    if (kind != kEntry) g.proj.push_back(r);
    ST_TRY(settle(e, s, false));
    if (s.refreshing) HIP_TRY(hipStreamWaitEvent(st, s.ev_ready, 0));
    ST_TRY(join(e, st));
    if (kind != kRow) ST_TRY(defer_flush(s, st));
    HIP_TRY(hipEventRecord(s.ev_u0, st));
    ST_TRY(run_groups(e, groups, st, false));
    if (s.angle) ST_TRY(run_tracks(e, {make_track(s, kind, payload)}, {(char)(s.esz == 8)}, st));
    HIP_TRY(hipEventRecord(s.ev_u1, st));
    s.have_update_time = true;
    if (kind == kRow) s.m += 1;
    if (kind == kCol) s.n += 1;
    s.t += 1;
    return after_update(e, s, st, nullptr);
}

// The engine's own streams (lanes, rotation lanes, refresh lanes).
std::vector<hipStream_t> engine_streams(isvd_engine* e) {
    std::vector<hipStream_t> v;
    for (hipStream_t q : {e->lane_a, e->lane_b, e->lane_c, e->rot_lane, e->rot_lane_b, e->capture_st})
        if (q) v.push_back(q);
    for (auto& l : e->rlanes)
        if (l.st) v.push_back(l.st);
    return v;
}

void bcache_drop_all(isvd_engine* e) {
    if (e->bcache.empty() && e->to_free.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto& kv : e->bcache) (void)hipFree(kv.second);
    e->bcache.clear();
    e->bcache_bytes = 0;
    for (char* p : e->to_free) (void)hipFree(p);
    e->to_free.clear();
}

// A block of at least `bytes` for a new stream whose work runs on `st`:
// a cached block no more than a quarter larger (st then waits for the engine
// streams as of the latest release), else a new allocation (after dropping
// the cache when the device is out of memory).
isvd_status release_poll(isvd_engine* e);
isvd_status block_alloc(isvd_engine* e, size_t bytes, hipStream_t st, char** out, size_t* got) {
    *out = nullptr;
    if (e->bcache_cap > 0) {
        ST_TRY(release_poll(e));
        auto it = e->bcache.lower_bound(bytes);
        if (it != e->bcache.end() && it->first <= bytes + bytes / 4) {
            *out = it->second;
            *got = it->first;
            e->bcache_bytes -= it->first;
            e->bcache.erase(it);
            for (hipEvent_t ev : e->ev_rel) HIP_TRY(hipStreamWaitEvent(st, ev, 0));
            return ISVD_OK;
        }
    }
    if (hipMalloc((void**)out, bytes) != hipSuccess) {
        (void)hipGetLastError();
        bcache_drop_all(e);
        if (hipMalloc((void**)out, bytes) != hipSuccess) {
            *out = nullptr;
            return fail(ISVD_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
        }
    }
    *got = bytes;
    return ISVD_OK;
}

void free_stream(isvd_engine* e, Stream* s) {
    if (!s) return;
    if (s->base) {
        (void)hipFree(s->base);
        e->used -= s->L.total;
    }
    if (s->slot >= 0) {
        e->hdr_free.push_back(s->slot);
        s->slot = -1;
        s->hdr = nullptr;
    }
    for (hipEvent_t* ev : {&s->ev_u0, &s->ev_u1, &s->ev_r0, &s->ev_r1, &s->ev_ready}) {
        if (*ev) (void)hipEventDestroy(*ev);
        *ev = nullptr;
    }
    if (s->wbuf) (void)hipFree(s->wbuf);
    s->wbuf = nullptr;
    if (s->a_host) (void)hipHostFree(s->a_host);
    s->a_host = nullptr;
    s->base = nullptr;
    s->live = false;
}

isvd_status validate_cfg(const isvd_config* c) {
    if (!c) return fail(ISVD_E_INVAL, "null config");
    if (c->m0 < 1 || c->n0 < 1) return fail(ISVD_E_INVAL, "empty A0 (%lld x %lld)", (long long)c->m0, (long long)c->n0);
    if (c->m_cap < c->m0 || c->n_cap < c->n0) return fail(ISVD_E_INVAL, "capacity below the initial shape");
    if (c->precision != ISVD_FP64 && c->precision != ISVD_FP32 && c->precision != ISVD_BF16ROT)
        return fail(ISVD_E_INVAL, "bad precision %d", c->precision);
    int kmax = std::max(c->k, c->policy.k_max);
    if (c->k < 1 || c->k > std::min<int64_t>(c->m0, c->n0) || kmax > kMaxRank)
        return fail(ISVD_E_INVAL, "k = %d outside [1, min(m0, n0, %d)]", c->k, kMaxRank);
    if (c->policy.kind < ISVD_POL_NONE || c->policy.kind > ISVD_POL_DRIFT)
        return fail(ISVD_E_INVAL, "bad policy kind %d", c->policy.kind);
    if (c->policy.kind == ISVD_POL_ANGLE && c->policy.angle_scope < 0)
        return fail(ISVD_E_INVAL, "negative angle scope");
    if (c->policy.kind == ISVD_POL_ADAPTIVE && (c->policy.k_max > 0 && c->policy.k_max < c->k))
        return fail(ISVD_E_INVAL, "adaptive rank: k_max %d below k %d", c->policy.k_max, c->k);
    return ISVD_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* isvd_last_error(void) { return g_err.c_str(); }

isvd_status isvd_engine_create(int32_t device, uint64_t hbm_budget_bytes, isvd_engine** out) {
    if (!out) return fail(ISVD_E_INVAL, "null output");
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(ISVD_E_INVAL, "device %d of %d", device, ndev);
    isvd_engine* e = new isvd_engine();
    e->device = device;
    e->budget = hbm_budget_bytes;
    isvd_status rc = ensure_device(e);
    if (rc == ISVD_OK) rc = set_lds_limits();
    if (rc == ISVD_OK) rc = noalloc_scratch_setup(device);
    if (rc == ISVD_OK) {
        e->ring.resize(64);
        for (Slot& s : e->ring) {
            if (hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) {
                rc = fail(ISVD_E_DEVICE, "event creation failed");
                break;
            }
        }
    }
    if (rc != ISVD_OK) {
        isvd_engine_destroy(e);
        return rc;
    }
    *out = e;
    return ISVD_OK;
}

isvd_status isvd_engine_destroy(isvd_engine* e) {
    if (!e) return ISVD_OK;
    (void)hipSetDevice(e->device);
    (void)hipDeviceSynchronize();
    for (Stream* s : e->streams) {
        free_stream(e, s);
        delete s;
    }
    for (Slot& s : e->ring)
        if (s.ev) (void)hipEventDestroy(s.ev);
    if (e->ring_host) (void)hipHostFree(e->ring_host);
    for (TickGraph* tg : e->tgraphs) free_tick_graph(tg);
    e->tgraphs.clear();
    if (e->capture_st) (void)hipStreamDestroy(e->capture_st);
    if (e->ring_dev) (void)hipFree(e->ring_dev);
    if (e->ws.p) (void)hipFree(e->ws.p);
    free_retired(e->ws);
    if (e->mws) (void)hipFree(e->mws);
    if (e->hdr_dev) (void)hipFree(e->hdr_dev);
    if (e->chain_plan) (void)hipFree(e->chain_plan);
    if (e->hdr_mirror) (void)hipHostFree(e->hdr_mirror);
    e->releasing.clear();   // their streams are freed with the others above
    for (char* p : e->to_free) (void)hipFree(p);
    e->to_free.clear();
    for (auto& kv : e->bcache) (void)hipFree(kv.second);
    e->bcache.clear();
    for (hipEvent_t ev : e->ev_rel) (void)hipEventDestroy(ev);
    if (e->seg_cws.p) (void)hipFree(e->seg_cws.p);
    free_retired(e->seg_cws);
    if (e->seg_cjobs.p) (void)hipFree(e->seg_cjobs.p);
    free_retired(e->seg_cjobs);
    if (e->chk_host) (void)hipHostFree(e->chk_host);
    for (auto& q : e->seg_slot) {
        if (q.host) (void)hipHostFree(q.host);
        if (q.ev) (void)hipEventDestroy(q.ev);
    }
    for (auto& l : e->rlanes) {
        if (l.ws.p) (void)hipFree(l.ws.p);
        free_retired(l.ws);
        if (l.jobs.p) (void)hipFree(l.jobs.p);
        free_retired(l.jobs);
        if (l.ev) (void)hipEventDestroy(l.ev);
        if (l.st) (void)hipStreamDestroy(l.st);
    }
    if (e->ev_policies) (void)hipEventDestroy(e->ev_policies);
    if (e->dsweeps) (void)hipFree(e->dsweeps);
    if (e->rsweeps) (void)hipHostFree(e->rsweeps);
    for (hipEvent_t ev : e->ev_pool) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : e->ev_core) (void)hipEventDestroy(ev);
    if (e->ev_main) (void)hipEventDestroy(e->ev_main);
    if (e->ev_fork) (void)hipEventDestroy(e->ev_fork);
    if (e->ev_b_end) (void)hipEventDestroy(e->ev_b_end);
    if (e->lane_b) (void)hipStreamDestroy(e->lane_b);
    if (e->lane_a) (void)hipStreamDestroy(e->lane_a);
    if (e->lane_c) (void)hipStreamDestroy(e->lane_c);
    if (e->ev_c_end) (void)hipEventDestroy(e->ev_c_end);
    if (e->ev_rot) (void)hipEventDestroy(e->ev_rot);
    for (hipEvent_t ev : e->ev_tick_end)
        if (ev) (void)hipEventDestroy(ev);
    if (e->rot_lane) (void)hipStreamDestroy(e->rot_lane);
    if (e->ev_rot_b) (void)hipEventDestroy(e->ev_rot_b);
    if (e->rot_lane_b) (void)hipStreamDestroy(e->rot_lane_b);
    delete e;
    return ISVD_OK;
}

isvd_status isvd_profile(isvd_engine* e, int32_t enable) {
    if (!e) return fail(ISVD_E_INVAL, "null engine");
    ST_TRY(ensure_device(e));
    if (enable) {
        HIP_TRY(hipDeviceSynchronize());
        e->prof.clear();
        e->ev_used = 0;
    }
    e->profiling = enable != 0;
    return ISVD_OK;
}

isvd_status isvd_sync(isvd_engine* e, void* hip_stream) {
    if (!e) return fail(ISVD_E_INVAL, "null engine");
    ST_TRY(ensure_device(e));
    ST_TRY(join_refreshes(e, (hipStream_t)hip_stream));
    return join(e, (hipStream_t)hip_stream);
}

isvd_status isvd_stream_busy(isvd_engine* e, isvd_id id, int32_t* busy) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    if (!busy) return fail(ISVD_E_INVAL, "null output");
    ST_TRY(ensure_device(e));
    ST_TRY(settle(e, *s, false));
    *busy = s->refreshing ? 1 : 0;
    return ISVD_OK;
}

isvd_status isvd_set_deferred_u(isvd_engine* e, int32_t enable, void* hip_stream) {
    if (!e) return fail(ISVD_E_INVAL, "null engine");
    ST_TRY(ensure_device(e));
    hipStream_t st = (hipStream_t)hip_stream;
    ST_TRY(join(e, st));
    for (Stream* s : e->streams) {
        if (!s || !s->live) continue;
        if (s->refreshing) HIP_TRY(hipStreamWaitEvent(st, s->ev_ready, 0));
        if (enable) {
            ST_TRY(ensure_wbuf(*s, st));
        } else {
            ST_TRY(defer_flush(*s, st));
        }
    }
    e->defer_u = enable != 0;
    return ISVD_OK;
}

isvd_status isvd_set_block_cache(isvd_engine* e, uint64_t bytes) {
    if (!e) return fail(ISVD_E_INVAL, "null engine");
    (void)hipSetDevice(e->device);
    e->bcache_cap = (size_t)bytes;
    if (e->bcache_bytes > e->bcache_cap) bcache_drop_all(e);
    return ISVD_OK;
}

isvd_status isvd_set_segmented_refresh(isvd_engine* e, int32_t enable) {
    if (!e) return fail(ISVD_E_INVAL, "null engine");
    e->seg_refresh = enable != 0;
    return ISVD_OK;
}

isvd_status isvd_set_tick_graphs(isvd_engine* e, int32_t enable) {
    if (!e) return fail(ISVD_E_INVAL, "null engine");
    ST_TRY(ensure_device(e));
    e->tick_graphs = enable != 0;
    if (!e->tick_graphs) {
        for (TickGraph* tg : e->tgraphs) free_tick_graph(tg);
        e->tgraphs.clear();
    }
    return ISVD_OK;
}

isvd_status isvd_set_pipelining(isvd_engine* e, int32_t enable) {
    if (!e) return fail(ISVD_E_INVAL, "null engine");
    e->pipelining = enable != 0;
    return ISVD_OK;
}

isvd_status isvd_rotation_stream(isvd_engine* e, void** out) {
    if (!e || !out) return fail(ISVD_E_INVAL, "null argument");
    ST_TRY(ensure_device(e));
    ST_TRY(ensure_lanes(e));
    *out = (void*)e->rot_lane;
    return ISVD_OK;
}

isvd_status isvd_set_rotation_variant(isvd_engine* e, int32_t kc, int32_t variant) {
    if (!e) return fail(ISVD_E_INVAL, "null engine");
    if (kc != 8 && kc != 16 && kc != 32 && kc != 64) return fail(ISVD_E_INVAL, "bucket %d is not tunable", kc);
    if (variant < 0 || variant >= kRotVariants) return fail(ISVD_E_INVAL, "variant %d not supported", variant);
    e->rot_var_f32[bucket_index(kc)] = variant;
    return ISVD_OK;
}

isvd_status isvd_autotune(isvd_engine* e, void* hip_stream, int32_t* variant_out, double* ms_out) {
    if (!e) return fail(ISVD_E_INVAL, "null engine");
    ST_TRY(ensure_device(e));
    hipStream_t st = (hipStream_t)hip_stream;
    const int nreq = 64;
    const int64_t m = 32768, n = 1024;
    const int kcs[4] = {8, 16, 32, 64};
    for (int bi = 0; bi < 4; ++bi) {
        const int kc = kcs[bi];
        // per request: U0, U1 (m x kc), V0, V1 (n x kc), QU, QV ((kc + 1) x kc), scratch
        const size_t ub = align_up(sizeof(float) * m * kc, 256), vb = align_up(sizeof(float) * n * kc, 256);
        const size_t qb = align_up(sizeof(float) * (kc + 1) * kc, 256), sb = align_up(sizeof(ReqScratch), 256);
        const size_t per = 2 * ub + 2 * vb + 2 * qb + sb;
        char* buf = nullptr;
        if (hipMalloc((void**)&buf, per * nreq) != hipSuccess) return fail(ISVD_E_NOMEM, "autotune buffers");
        auto cleanup = [&]() { (void)hipFree(buf); };
        const int64_t nfl = (int64_t)(per * nreq / sizeof(float));
        k_fill_hash<<<(int)std::min<int64_t>(cdiv(nfl, 256), 65535), 256, 0, st>>>((float*)buf, nfl, 0x9e37u + kc);
        std::vector<ReqScratch> scr(nreq);
        std::vector<Req> reqs(nreq);
        for (int q = 0; q < nreq; ++q) {
            char* b = buf + per * q;
            ReqScratch& r = scr[q];
            r.skip = 0;
            r.k_in = r.ld_in = r.k_out = r.ld_out = kc;
            r.in_idx = 0;
            r.inv_rho = 0.0;
            Req& rq = reqs[q];
            rq = Req{};
            rq.m = m;
            rq.n = n;
            rq.kind = kEntry;
            rq.U[0] = b;
            rq.U[1] = b + ub;
            rq.V[0] = b + 2 * ub;
            rq.V[1] = b + 2 * ub + vb;
            rq.QU = b + 2 * ub + 2 * vb;
            rq.QV = b + 2 * ub + 2 * vb + qb;
            rq.rs = (ReqScratch*)(b + 2 * ub + 2 * vb + 2 * qb);
        }
        for (int q = 0; q < nreq; ++q)
            if (hipMemcpyAsync(reqs[q].rs, &scr[q], sizeof(ReqScratch), hipMemcpyHostToDevice, st) != hipSuccess) {
                cleanup();
                return fail(ISVD_E_DEVICE, "autotune upload");
            }
        double best = 1e30;
        int best_var = e->rot_var_f32[bi];
        for (int ci = 0; ci < kRotVariants; ++ci) {
            Group g{};
            g.fp64 = false;
            g.kc = kc;
            g.var = ci;
            g.rows = kRotVariant[ci].rows;
            for (Req rq : reqs) {
                rq.rot_tiles_u = (int)cdiv(m, g.rows);
                g.all.push_back(rq);
            }
            g.pre_proj.assign(1, 0);
            g.pre_rot.assign(nreq + 1, 0);
            for (int q = 0; q < nreq; ++q) g.pre_rot[q + 1] = g.pre_rot[q] + rot_tiles(g.all[q], g.rows);
            const size_t off_all = 0, off_pr = align_up(sizeof(Req) * nreq, 64);
            const size_t bytes = off_pr + sizeof(int) * (nreq + 1);
            g.off_all = off_all;
            g.off_pr = off_pr;
            Slot* slot = nullptr;
            isvd_status rc = acquire_slot(e, bytes, &slot);
            if (rc != ISVD_OK) { cleanup(); return rc; }
            memcpy(slot->host + off_all, g.all.data(), sizeof(Req) * nreq);
            memcpy(slot->host + off_pr, g.pre_rot.data(), sizeof(int) * (nreq + 1));
            hipEvent_t e0, e1;
            if (hipMemcpyAsync(slot->dev, slot->host, bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
                hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
                cleanup();
                return fail(ISVD_E_DEVICE, "autotune launch set-up");
            }
            const int reps = 6;
            for (int w = 0; w < 2; ++w) rc = launch_phase(g, slot->dev, 5, st);
            (void)hipEventRecord(e0, st);
            for (int w = 0; w < reps && rc == ISVD_OK; ++w) rc = launch_phase(g, slot->dev, 5, st);
            (void)hipEventRecord(e1, st);
            (void)hipEventRecord(slot->ev, st);
            slot->used = true;
            float ms = 0.f;
            if (rc == ISVD_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = fail(ISVD_E_DEVICE, "autotune timing");
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            if (rc != ISVD_OK) { cleanup(); return rc; }
            const double per_launch = ms / reps;
            if (ms_out) ms_out[bi * kRotVariants + ci] = per_launch;
            // a later shape must win by 3%: near-equal shapes resolve to the
            // earlier one, so repeated tunings on one device agree
            if (per_launch < (ci == 0 ? best : 0.97 * best)) { best = per_launch; best_var = ci; }
        }
        HIP_TRY(hipStreamSynchronize(st));
        cleanup();
        e->rot_var_f32[bi] = best_var;
        if (variant_out) variant_out[bi] = best_var;
    }
    return ISVD_OK;
}

isvd_status isvd_profile_read(isvd_engine* e, isvd_launch_time* out, int32_t cap, int32_t* count) {
    if (!e || !count || (cap > 0 && !out)) return fail(ISVD_E_INVAL, "null argument");
    ST_TRY(ensure_device(e));
    *count = (int32_t)e->prof.size();
    for (int32_t q = 0; q < cap && q < (int32_t)e->prof.size(); ++q) {
        const LaunchRec& r = e->prof[q];
        HIP_TRY(hipEventSynchronize(r.e));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.b, r.e));
        out[q].phase = r.phase;
        out[q].kc = r.kc;
        out[q].fp64 = r.fp64;
        out[q].nreq = r.nreq;
        out[q].blocks = r.blocks;
        out[q].ms = ms;
    }
    return ISVD_OK;
}

uint64_t isvd_stream_bytes(const isvd_config* cfg) {
    if (validate_cfg(cfg) != ISVD_OK) return 0;
    int64_t nt = 0;
    int kc = bucket_for(round4(std::max(cfg->k, cfg->policy.k_max)));
    Layout L = make_layout(*cfg, cfg->precision == ISVD_FP64 ? 8 : 4, kc, &nt);
    return L.total;
}

struct GivenFactors {
    const double *U, *S, *V;
    int64_t ldu, ldv;
};

static isvd_status install_factors(Stream& s, const GivenFactors& f, hipStream_t st) {
    const int k = s.k_target, ld = round4(k);
    const int64_t m = s.m, n = s.n;
    // tiled basis layout, whole tiles, zero padding
    std::vector<char> bu((size_t)s.esz * round16(m) * ld, 0), bv((size_t)s.esz * round16(n) * ld, 0);
    for (int64_t r = 0; r < m; ++r)
        for (int c = 0; c < k; ++c) {
            if (s.esz == 8) ((double*)bu.data())[uvo(r, c, ld)] = f.U[r * f.ldu + c];
            else ((float*)bu.data())[uvo(r, c, ld)] = (float)f.U[r * f.ldu + c];
        }
    for (int64_t r = 0; r < n; ++r)
        for (int c = 0; c < k; ++c) {
            if (s.esz == 8) ((double*)bv.data())[uvo(r, c, ld)] = f.V[r * f.ldv + c];
            else ((float*)bv.data())[uvo(r, c, ld)] = (float)f.V[r * f.ldv + c];
        }
    HIP_TRY(hipMemcpyAsync(s.U[1], bu.data(), bu.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s.V[1], bv.data(), bv.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s.Uref, bu.data(), bu.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s.S, f.S, sizeof(double) * k, hipMemcpyHostToDevice, st));
    k_set_header<<<1, 1, 0, st>>>(s.hdr, k, ld, 1, 0);
    k_sigma_trackers<<<1, 1, 0, st>>>(s.hdr, s.S, k);
    k_track_reset<<<1, kThreads, 0, st>>>(s.hdr, s.TM, s.TH, s.kc);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return ISVD_OK;
}

static isvd_status init_common(isvd_engine* e, const isvd_config* cfg, const void* A0, int64_t lda, int32_t dtype,
                               int32_t on_device, const GivenFactors* given, void* hip_stream, isvd_id* out,
                               std::vector<Stream*>* batch = nullptr) {
    if (!e || !out) return fail(ISVD_E_INVAL, "null engine or output");
    ST_TRY(validate_cfg(cfg));
    if (!A0) return fail(ISVD_E_INVAL, "null A0");
    if (lda < cfg->n0) return fail(ISVD_E_INVAL, "lda %lld < n0 %lld", (long long)lda, (long long)cfg->n0);
    if (dtype != ISVD_DTYPE_F32 && dtype != ISVD_DTYPE_F64) return fail(ISVD_E_INVAL, "bad dtype %d", dtype);
    ST_TRY(ensure_device(e));
    hipStream_t st = (hipStream_t)hip_stream;
    Stream* s = new Stream();
    s->cfg = *cfg;
    if (s->cfg.tol_rel <= 0.0) s->cfg.tol_rel = cfg->precision == ISVD_FP64 ? 1e-10 : 1e-5;
    s->esz = cfg->precision == ISVD_FP64 ? 8 : 4;
    s->bf16 = cfg->precision == ISVD_BF16ROT;
    s->kc = bucket_for(round4(std::max(cfg->k, cfg->policy.k_max)));
    s->k_target = cfg->k;
    s->angle = cfg->policy.kind == ISVD_POL_ANGLE;
    s->m = cfg->m0;
    s->n = cfg->n0;
    s->L = make_layout(s->cfg, s->esz, s->kc, &s->ntiles_max);
    if (e->budget && e->used + s->L.total > e->budget) {
        const size_t bytes = s->L.total;
        delete s;
        return fail(ISVD_E_BUDGET, "stream needs %zu bytes, %llu of %llu in use", bytes,
                    (unsigned long long)e->used, (unsigned long long)e->budget);
    }
    if (!e->hdr_dev) {
        if (hipMalloc((void**)&e->hdr_dev, sizeof(DevHeader) * kMaxLiveStreams) != hipSuccess ||
            hipHostMalloc((void**)&e->hdr_mirror, sizeof(DevHeader) * kMaxLiveStreams, hipHostMallocDefault) !=
                hipSuccess) {
            delete s;
            return fail(ISVD_E_NOMEM, "stream header array");
        }
    }
    if (e->hdr_free.empty() && e->hdr_hi >= kMaxLiveStreams) {
        delete s;
        return fail(ISVD_E_NOMEM, "more than %d live streams", kMaxLiveStreams);
    }
    {
        isvd_status rc = block_alloc(e, s->L.total, st, &s->base, &s->base_bytes);
        if (rc != ISVD_OK) {
            s->base = nullptr;
            delete s;
            return rc;
        }
    }
    e->used += s->L.total;
    char* b = s->base;
    if (!e->hdr_free.empty()) {
        s->slot = e->hdr_free.back();
        e->hdr_free.pop_back();
    } else {
        s->slot = e->hdr_hi++;
    }
    s->hdr = e->hdr_dev + s->slot;
    for (int q = 0; q < 2; ++q) {
        s->rs[q] = (ReqScratch*)(b + s->L.rs + q * s->L.rs_b);
        s->p[q] = (double*)(b + s->L.p + q * s->L.p_b);
        s->QU[q] = b + s->L.QU + q * s->L.q_b;
        s->QV[q] = b + s->L.QV + q * s->L.q_b;
    }
    s->S = (double*)(b + s->L.S);
    s->partials = (double*)(b + s->L.partials);
    s->partials2 = (double*)(b + s->L.partials2);
    s->stage = b + s->L.stage;
    s->U[0] = b + s->L.U0;
    s->U[1] = b + s->L.U1;
    s->V[0] = b + s->L.V0;
    s->V[1] = b + s->L.V1;
    s->Uref = b + s->L.Uref;
    if (cfg->policy.kind == ISVD_POL_ANGLE) {
        s->TM = (double*)(b + s->L.TM);
        s->TH = (double*)(b + s->L.TH);
        s->TP = (double*)(b + s->L.TP);
        s->TS = (double*)(b + s->L.TS);
    }
    if (core_jg_doubles(s->kc) > 0 && s->esz == 8) s->Jg = (double*)(b + s->L.Jg);
    if (cfg->a_on_host) {
        if (hipHostMalloc(&s->a_host, s->L.a_bytes, hipHostMallocDefault) != hipSuccess) {
            s->a_host = nullptr;
            free_stream(e, s);
            delete s;
            return fail(ISVD_E_NOMEM, "pinned host A of %zu bytes", s->L.a_bytes);
        }
        std::memset(s->a_host, 0, s->L.a_bytes);
        void* dptr = nullptr;
        if (hipHostGetDevicePointer(&dptr, s->a_host, 0) != hipSuccess) {
            free_stream(e, s);
            delete s;
            return fail(ISVD_E_DEVICE, "device view of the host A");
        }
        s->A = (char*)dptr;
    } else {
        s->A = b + s->L.A;
    }
    s->live = true;
    e->streams.push_back(s);
    const isvd_id id = (isvd_id)e->streams.size() - 1;
    auto bail = [&](isvd_status rc) {
        free_stream(e, s);
        return rc;
    };
    if (hipEventCreateWithFlags(&s->ev_ready, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&s->ev_u0) != hipSuccess || hipEventCreate(&s->ev_u1) != hipSuccess ||
        hipEventCreate(&s->ev_r0) != hipSuccess || hipEventCreate(&s->ev_r1) != hipSuccess)
        return bail(fail(ISVD_E_DEVICE, "event creation failed"));
    DevHeader h0{};
    h0.k = 0;
    h0.ld = 4;
    h0.m = cfg->m0;
    h0.n = cfg->n0;
    // A is zeroed whole: entries outside the current m x n stay zero (the
    // refresh products read the padding columns of a row)
    if (hipMemsetAsync(s->base, 0, s->L.U0, st) != hipSuccess ||
        (!cfg->a_on_host && hipMemsetAsync(s->A, 0, s->L.a_bytes, st) != hipSuccess) ||
        hipMemcpyAsync(s->hdr, &h0, sizeof(h0), hipMemcpyHostToDevice, st) != hipSuccess)
        return bail(fail(ISVD_E_DEVICE, "header initialisation failed"));
    // A_0 into A (leading dimension lda_of), converting to the storage type
    const int64_t m0 = cfg->m0, n0 = cfg->n0, ldA = lda_of(*cfg);
    const int64_t cnt = m0 * n0;
    const void* src = A0;
    void* tmpdev = nullptr;
    if (!on_device) {
        size_t bytes = (size_t)(dtype == ISVD_DTYPE_F64 ? 8 : 4) * m0 * lda;
        if (hipMalloc(&tmpdev, bytes) != hipSuccess) return bail(fail(ISVD_E_NOMEM, "A0 staging"));
        if (hipMemcpyAsync(tmpdev, A0, bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
            (void)hipFree(tmpdev);
            return bail(fail(ISVD_E_DEVICE, "A0 upload"));
        }
        src = tmpdev;
    }
    const int blocks = (int)cdiv(cnt, 256);
    if (dtype == ISVD_DTYPE_F64 && s->esz == 8)
        k_copy2d<double, double><<<blocks, 256, 0, st>>>((const double*)src, lda, (double*)s->A, ldA, m0, n0);
    else if (dtype == ISVD_DTYPE_F64)
        k_copy2d<double, float><<<blocks, 256, 0, st>>>((const double*)src, lda, (float*)s->A, ldA, m0, n0);
    else if (s->esz == 8)
        k_copy2d<float, double><<<blocks, 256, 0, st>>>((const float*)src, lda, (double*)s->A, ldA, m0, n0);
    else
        k_copy2d<float, float><<<blocks, 256, 0, st>>>((const float*)src, lda, (float*)s->A, ldA, m0, n0);
    if (hipGetLastError() != hipSuccess) return bail(fail(ISVD_E_DEVICE, "A0 copy launch"));
    // N_0 = ||A_0||_F^2 (sum of per-chunk partials, FP64)
    const size_t fro_bytes = sizeof(double) * (size_t)cdiv(m0, kFroRows);
    isvd_status rc = ensure_ws(e, std::max(fro_bytes, (size_t)4096));
    if (rc != ISVD_OK) return bail(rc);
    const int nchunk = (int)cdiv(m0, kFroRows);
    if (s->esz == 8)
        k_fro2_partial<double><<<nchunk, kThreads, 0, st>>>((const double*)s->A, ldA, m0, n0, (double*)e->ws.p);
    else
        k_fro2_partial<float><<<nchunk, kThreads, 0, st>>>((const float*)s->A, ldA, m0, n0, (double*)e->ws.p);
    k_sum_block<<<1, kThreads, 0, st>>>((const double*)e->ws.p, nchunk, &s->hdr->N);
    if (hipGetLastError() != hipSuccess) return bail(fail(ISVD_E_DEVICE, "norm launch"));
    if (e->defer_u) {
        rc = ensure_wbuf(*s, st);
        if (rc != ISVD_OK) return bail(rc);
    }
    if (given)
        rc = install_factors(*s, *given, st);
    else if (batch && e->seg_refresh && seg_eligible(*s))
        batch->push_back(s);   // the caller runs the batch's initial SVDs together
    else
        rc = init_on_lane(e, *s, st);
    if (tmpdev) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(tmpdev);
    }
    if (rc != ISVD_OK) return bail(rc);
    *out = id;
    return ISVD_OK;
}

isvd_status isvd_init(isvd_engine* e, const isvd_config* cfg, const void* A0, int64_t lda, int32_t dtype,
                      int32_t on_device, void* hip_stream, isvd_id* out) {
    return init_common(e, cfg, A0, lda, dtype, on_device, nullptr, hip_stream, out);
}

isvd_status isvd_init_batch(isvd_engine* e, int32_t count, const isvd_config* cfgs, const void* const* A0,
                            const int64_t* lda, const int32_t* dtype, void* hip_stream, isvd_id* ids,
                            int32_t* created) {
    if (!e || count < 0 || (count > 0 && (!cfgs || !A0 || !lda || !dtype || !ids)))
        return fail(ISVD_E_INVAL, "null argument");
    if (created) *created = 0;
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<Stream*> batch;
    isvd_status rc = ISVD_OK;
    int32_t q = 0;
    for (; q < count; ++q) {
        rc = init_common(e, &cfgs[q], A0[q], lda[q], dtype[q], 1, nullptr, hip_stream, &ids[q], &batch);
        if (rc != ISVD_OK) break;
    }
    // the batched initial SVDs on the next refresh lane in turn, after the copies of A_0 on st
    if (!batch.empty()) {
        isvd_status rb = ensure_refresh_lanes(e);
        if (rb == ISVD_OK) {
            auto& lane = e->rlanes[e->seg_lane];
            e->seg_lane = (e->seg_lane + 1) % kRefreshLanes;
            if (hipEventRecord(e->ev_policies, st) != hipSuccess ||
                hipStreamWaitEvent(lane.st, e->ev_policies, 0) != hipSuccess)
                rb = fail(ISVD_E_DEVICE, "batch ordering failed");
            if (rb == ISVD_OK) rb = refresh_segmented(e, batch, lane, true);
            if (rb == ISVD_OK && hipEventRecord(lane.ev, lane.st) != hipSuccess)
                rb = fail(ISVD_E_DEVICE, "batch event failed");
            lane.pending = true;
        }
        if (rb != ISVD_OK) {
            // leave no stream without its initial SVD: release every stream of the call
            for (int32_t i = 0; i < q; ++i) {
                (void)isvd_release(e, ids[i]);
                ids[i] = -1;
            }
            return rb;
        }
    }
    if (created) *created = q;
    return rc;
}

isvd_status isvd_init_from_factors(isvd_engine* e, const isvd_config* cfg, const void* A0, int64_t lda,
                                   int32_t dtype, int32_t on_device, const double* U, int64_t ldu,
                                   const double* S, const double* V, int64_t ldv, void* hip_stream,
                                   isvd_id* out) {
    if (!cfg || !U || !S || !V || ldu < cfg->k || ldv < cfg->k) return fail(ISVD_E_INVAL, "bad factor arguments");
    for (int q = 0; q < cfg->k; ++q)
        if (!(S[q] >= 0.0) || (q > 0 && S[q] > S[q - 1])) return fail(ISVD_E_INVAL, "S must be non-increasing and >= 0");
    GivenFactors f{U, S, V, ldu, ldv};
    return init_common(e, cfg, A0, lda, dtype, on_device, &f, hip_stream, out);
}

isvd_status isvd_append_row(isvd_engine* e, isvd_id id, const void* x, int64_t n, int32_t dtype,
                            int32_t on_device, void* hip_stream) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    if (n != s->n) return fail(ISVD_E_SHAPE, "row of length %lld, stream has n = %lld", (long long)n, (long long)s->n);
    if (s->m >= s->cfg.m_cap) return fail(ISVD_E_CAPACITY, "row capacity %lld reached", (long long)s->cfg.m_cap);
    ST_TRY(ensure_device(e));
    hipStream_t st = (hipStream_t)hip_stream;
    const void* pay = nullptr;
    ST_TRY(stage_payload(*s, x, n, dtype, on_device, st, &pay));
    return single_update(e, *s, kRow, pay, 0, 0, 0.0, st);
}

isvd_status isvd_append_col(isvd_engine* e, isvd_id id, const void* y, int64_t m, int32_t dtype,
                            int32_t on_device, void* hip_stream) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    if (m != s->m) return fail(ISVD_E_SHAPE, "column of length %lld, stream has m = %lld", (long long)m, (long long)s->m);
    if (s->n >= s->cfg.n_cap) return fail(ISVD_E_CAPACITY, "column capacity %lld reached", (long long)s->cfg.n_cap);
    ST_TRY(ensure_device(e));
    hipStream_t st = (hipStream_t)hip_stream;
    const void* pay = nullptr;
    ST_TRY(stage_payload(*s, y, m, dtype, on_device, st, &pay));
    return single_update(e, *s, kCol, pay, 0, 0, 0.0, st);
}

isvd_status isvd_update_entry(isvd_engine* e, isvd_id id, int64_t i, int64_t j, double delta, void* hip_stream) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    if (i < 0 || i >= s->m || j < 0 || j >= s->n)
        return fail(ISVD_E_RANGE, "entry (%lld, %lld) outside %lld x %lld", (long long)i, (long long)j,
                    (long long)s->m, (long long)s->n);
    if (!std::isfinite(delta)) return fail(ISVD_E_NONFINITE, "delta is not finite");
    ST_TRY(ensure_device(e));
    return single_update(e, *s, kEntry, nullptr, i, j, delta, (hipStream_t)hip_stream);
}

isvd_status isvd_refresh(isvd_engine* e, isvd_id id, int32_t store_reference, void* hip_stream) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    ST_TRY(ensure_device(e));
    ST_TRY(settle(e, *s, true));
    ST_TRY(join(e, (hipStream_t)hip_stream));
    return do_refresh(e, *s, false, store_reference != 0, (hipStream_t)hip_stream);
}

isvd_status isvd_refresh_noalloc(isvd_engine* e, isvd_id id, int32_t store_reference, void* hip_stream) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    ST_TRY(ensure_device(e));
    char* base = (e->device >= 0 && e->device < kMaxDevices) ? g_scratch_ptr[e->device] : nullptr;
    if (!base) return fail(ISVD_E_DEVICE, "no allocation-free scratch on device %d", e->device);
    if (!store_reference && s->TM)
        return fail(ISVD_E_INVAL, "keeping the old reference of an angle-policy stream needs tracker workspace, "
                                  "which only isvd_refresh allocates");
    int k = 0, b = 0;
    refresh_block(*s, &k, &b);
    if (b < k) return fail(ISVD_E_INVAL, "refresh block %d smaller than rank %d", b, k);
    const WsLayout w = ws_layout(s->m, s->n, b, s->esz);
    const size_t need = gram_form(*s, b) ? gcf_layout(s->m, s->n, w.total, kNoAllocScratchBytes).total : w.total;
    if (need > kNoAllocScratchBytes)
        return fail(ISVD_E_NOMEM, "the refresh of a %lld x %lld stream needs %zu bytes of workspace; the "
                                  "allocation-free scratch holds %zu",
                    (long long)s->m, (long long)s->n, need, kNoAllocScratchBytes);
    ST_TRY(settle(e, *s, true));
    ST_TRY(join(e, (hipStream_t)hip_stream));
    WsBuf wk;
    wk.p = base;
    wk.bytes = kNoAllocScratchBytes;
    wk.fixed = true;
    return do_refresh(e, *s, false, store_reference != 0, (hipStream_t)hip_stream, nullptr, nullptr, nullptr, &wk);
}

isvd_status isvd_metrics(isvd_engine* e, isvd_id id, int32_t compute_exact, void* hip_stream, isvd_metrics_t* out) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    if (!out) return fail(ISVD_E_INVAL, "null output");
    ST_TRY(ensure_device(e));
    hipStream_t st = (hipStream_t)hip_stream;
    ST_TRY(settle(e, *s, true));
    ST_TRY(join(e, st));
    if (compute_exact) ST_TRY(defer_flush(*s, st));
    DevHeader h{};
    std::vector<double> S(s->kc + 2, 0.0);
    HIP_TRY(hipMemcpyAsync(&h, s->hdr, sizeof(h), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(S.data(), s->S, sizeof(double) * S.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h.status != 0) {
        // a request was rejected on the device: report it once, adopt the
        // device's shape and tick count, and re-open the stream
        s->m = h.m;
        s->n = h.n;
        s->t = h.t;
        const int32_t zero = 0;
        HIP_TRY(hipMemcpyAsync((char*)s->hdr + offsetof(DevHeader, status), &zero, sizeof(zero),
                               hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    const double nan = std::nan("");
    isvd_metrics_t m{};
    m.t = h.t;
    m.m = h.m;
    m.n = h.n;
    m.n_refresh = s->n_refresh;
    m.t_last_refresh = s->t_last;
    m.n_rejected = h.n_rejected;
    m.k = h.k;
    m.status = h.status;
    m.sweeps = h.sweeps;
    m.new_direction = h.new_dir;
    m.fro2_A = h.N;
    double s2 = 0.0;
    for (int q = 0; q < h.k; ++q) s2 += S[q] * S[q];
    m.sigma2_sum = s2;
    m.evr = h.N > 0.0 ? s2 / h.N : nan;
    m.rho = h.rho;
    m.novelty = h.novelty;
    m.step_angle_U = h.t > 0 ? h.step_angle_u : nan;
    m.step_angle_V = h.t > 0 ? h.step_angle_v : nan;
    m.spectrum_change = h.t > 0 ? h.spec_change : nan;
    m.refresh_rounds = s->refresh_rounds;
    m.refresh_converged = s->refresh_converged ? 1 : 0;
    m.drift_U = s->cfg.policy.kind == ISVD_POL_DRIFT ? s->drift_acc : nan;
    m.frob_error = m.frob_opt = m.frob_gap = m.frob_ratio = nan;
    m.ortho_U = m.ortho_V = nan;
    m.angle_opt = nan;
    m.angle_ref = s->angle ? h.angle_ref : nan;
    m.update_time_us = nan;
    m.opt_time_us = nan;
    float ms = 0.f;
    if (s->have_update_time && hipEventElapsedTime(&ms, s->ev_u0, s->ev_u1) == hipSuccess) m.update_time_us = 1e3 * ms;
    if (s->have_refresh_time && hipEventElapsedTime(&ms, s->ev_r0, s->ev_r1) == hipSuccess) m.opt_time_us = 1e3 * ms;
    if (compute_exact) {
        Exact ex;
        RefreshPlan plan;
        ST_TRY(exact_metrics(e, *s, st, &ex, &plan));
        m.frob_error = ex.e_inc;
        m.frob_opt = ex.e_opt;
        m.frob_gap = ex.gap;
        m.frob_ratio = ex.ratio;
        m.ortho_U = ex.ortho_u;
        m.ortho_V = ex.ortho_v;
        m.angle_opt = ex.angle_opt;
        ST_TRY(direct_trackers(e, *s, st, &m.angle_ref, nullptr, nullptr, 0));
    }
    *out = m;
    return ISVD_OK;
}

isvd_status isvd_causal_center(const void* r, void* out, int64_t rows, int64_t n, int32_t dtype, double* mu,
                               int64_t t0, void* hip_stream) {
    if (!r || !out || !mu) return fail(ISVD_E_INVAL, "null rows, output or mean");
    if (rows < 1 || n < 1 || t0 < 0) return fail(ISVD_E_INVAL, "rows %lld, n %lld, t0 %lld", (long long)rows,
                                                 (long long)n, (long long)t0);
    if (dtype != ISVD_DTYPE_F32 && dtype != ISVD_DTYPE_F64) return fail(ISVD_E_INVAL, "bad dtype %d", dtype);
    hipStream_t st = (hipStream_t)hip_stream;
    const int blocks = (int)cdiv(n, 256);
    if (dtype == ISVD_DTYPE_F64)
        k_causal_center<double><<<blocks, 256, 0, st>>>((const double*)r, (double*)out, rows, n, mu, t0);
    else
        k_causal_center<float><<<blocks, 256, 0, st>>>((const float*)r, (float*)out, rows, n, mu, t0);
    HIP_TRY(hipGetLastError());
    return ISVD_OK;
}

isvd_status isvd_covariance(isvd_engine* e, isvd_id id, double* cov, int64_t ldc, void* hip_stream) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    if (!cov) return fail(ISVD_E_INVAL, "null covariance buffer");
    ST_TRY(ensure_device(e));
    hipStream_t st = (hipStream_t)hip_stream;
    // after the stream's queued work (a lane refresh, pending U rotations) on
    // the GPU; the kernel reads rank and buffer from the device header
    if (s->refreshing) HIP_TRY(hipStreamWaitEvent(st, s->ev_ready, 0));
    ST_TRY(join(e, st));
    const int64_t n = s->n;
    if (ldc < n) return fail(ISVD_E_INVAL, "ldc %lld < n %lld", (long long)ldc, (long long)n);
    if (s->m < 2) return fail(ISVD_E_INVAL, "covariance needs at least two rows");
    dim3 grid((unsigned)cdiv(n, kCovTile), (unsigned)cdiv(n, kCovTile));
    if (s->esz == 8)
        k_lowrank_cov<double><<<grid, 256, 0, st>>>(s->hdr, (const double*)s->V[0], (const double*)s->V[1], s->S, n,
                                                    cov, ldc);
    else
        k_lowrank_cov<float><<<grid, 256, 0, st>>>(s->hdr, (const float*)s->V[0], (const float*)s->V[1], s->S, n,
                                                   cov, ldc);
    HIP_TRY(hipGetLastError());
    return ISVD_OK;
}

}  // extern "C"

namespace {
template <typename T>
isvd_status risk_t(isvd_engine* e, Stream& s, const DevHeader& h, const double* w, bool exact, isvd_risk_t* out,
                   hipStream_t st) {
    const int64_t n = h.n;
    const int k = h.k;
    const double inv_t1 = 1.0 / (double)(h.m - 1);
    // device scratch: w, y_inc, y_full, G_inc, G_full, C, then V_full (tiled)
    const int kf_max = kMaxCore;
    const size_t nd = (size_t)n + 2 * kf_max + 3 * (size_t)kf_max * kf_max;
    const size_t vf_off = align_up(sizeof(double) * nd, 256);
    const size_t vf_bytes = (size_t)s.esz * round16(n) * round4(kf_max);
    ST_TRY(ensure_mws(e, vf_off + (exact ? vf_bytes : 0)));
    double* dw = (double*)e->mws;
    double* y_inc = dw + n;
    double* y_full = y_inc + kf_max;
    double* G_inc = y_full + kf_max;
    double* G_full = G_inc + kf_max * kf_max;
    double* Cx = G_full + kf_max * kf_max;
    T* Vf = (T*)(e->mws + vf_off);
    const T* Vi = (const T*)s.V[h.cur];
    HIP_TRY(hipMemcpyAsync(dw, w, sizeof(double) * n, hipMemcpyHostToDevice, st));
    k_vt_w<T><<<k, 256, 0, st>>>(Vi, h.ld, n, dw, y_inc);
    HIP_TRY(hipGetLastError());
    std::vector<double> si(k), yi(k);
    HIP_TRY(hipMemcpyAsync(si.data(), s.S, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(yi.data(), y_inc, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    const double nan = std::nan("");
    out->vol_full = out->err_risk = out->err_cov = nan;
    if (!exact) {
        HIP_TRY(hipStreamSynchronize(st));
    } else {
        // TruncatedSVD(A_t, k): the refresh's computation, V_full = X H as the
        // refresh would commit it, but into scratch (the stream is unchanged)
        RefreshPlan plan;
        ST_TRY(refresh_compute<T>(e, s, false, st, &plan));
        const char* ws = e->ws.p;
        const int kf = plan.k;
        k_rotate_plain<T, 128, true><<<(int)cdiv(plan.n, 16), kThreads, 0, st>>>(
            (const T*)(ws + plan.w.X), plan.b, Vf, plan.ldo, plan.n, plan.b, (const T*)(ws + plan.w.QV));
        k_vt_w<T><<<kf, 256, 0, st>>>(Vf, plan.ldo, n, dw, y_full);
        k_cross<T, T><<<k, 128, 0, st>>>(Vi, h.ld, Vi, h.ld, n, k, G_inc);
        k_cross<T, T><<<kf, 128, 0, st>>>(Vf, plan.ldo, Vf, plan.ldo, n, kf, G_full);
        k_cross<T, T><<<k, 128, 0, st>>>(Vi, h.ld, Vf, plan.ldo, n, kf, Cx);
        HIP_TRY(hipGetLastError());
        std::vector<double> sf(kf), yf(kf), gi((size_t)k * k), gf((size_t)kf * kf), cx((size_t)k * kf);
        int sweeps = 0;
        HIP_TRY(hipMemcpyAsync(sf.data(), ws + plan.w.Sr, sizeof(double) * kf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(yf.data(), y_full, sizeof(double) * kf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(gi.data(), G_inc, sizeof(double) * gi.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(gf.data(), G_full, sizeof(double) * gf.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(cx.data(), Cx, sizeof(double) * cx.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&sweeps, ws + plan.w.sweeps, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (sweeps < 0) return fail(ISVD_E_CONVERGE, "Rayleigh-Ritz Jacobi did not converge");
        double vf2 = 0.0, nf2 = 0.0, ni2 = 0.0, x2 = 0.0;
        for (int c = 0; c < kf; ++c) vf2 += sf[c] * sf[c] * inv_t1 * yf[c] * yf[c];
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                const double g = gi[(size_t)i * k + j];
                ni2 += (si[i] * si[i] * inv_t1) * (si[j] * si[j] * inv_t1) * g * g;
            }
        for (int i = 0; i < kf; ++i)
            for (int j = 0; j < kf; ++j) {
                const double g = gf[(size_t)i * kf + j];
                nf2 += (sf[i] * sf[i] * inv_t1) * (sf[j] * sf[j] * inv_t1) * g * g;
            }
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < kf; ++j) {
                const double c = cx[(size_t)i * kf + j];
                x2 += (si[i] * si[i] * inv_t1) * (sf[j] * sf[j] * inv_t1) * c * c;
            }
        out->vol_full = std::sqrt(std::max(vf2, 0.0));
        out->err_cov = nf2 > 0.0 ? std::sqrt(std::max(ni2 + nf2 - 2.0 * x2, 0.0)) / std::sqrt(nf2) : nan;
    }
    double vi2 = 0.0;
    for (int c = 0; c < k; ++c) vi2 += si[c] * si[c] * inv_t1 * yi[c] * yi[c];
    out->vol_inc = std::sqrt(std::max(vi2, 0.0));
    if (exact) out->err_risk = out->vol_full > 0.0 ? std::fabs(out->vol_inc - out->vol_full) / out->vol_full : nan;
    return ISVD_OK;
}
}  // namespace

extern "C" {

isvd_status isvd_risk(isvd_engine* e, isvd_id id, const double* w, int64_t n, int32_t exact, isvd_risk_t* out,
                      void* hip_stream) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    if (!w || !out) return fail(ISVD_E_INVAL, "null weights or output");
    ST_TRY(ensure_device(e));
    hipStream_t st = (hipStream_t)hip_stream;
    ST_TRY(settle(e, *s, true));
    ST_TRY(join(e, st));
    DevHeader h{};
    ST_TRY(read_header(*s, st, &h));
    if (n != h.n) return fail(ISVD_E_SHAPE, "weights length %lld != n %lld", (long long)n, (long long)h.n);
    if (h.m < 2) return fail(ISVD_E_INVAL, "volatility needs at least two rows");
    return s->esz == 8 ? risk_t<double>(e, *s, h, w, exact != 0, out, st)
                       : risk_t<float>(e, *s, h, w, exact != 0, out, st);
}

isvd_status isvd_get_factors(isvd_engine* e, isvd_id id, double* U, int64_t ldu, double* S, double* V, int64_t ldv,
                             void* hip_stream) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    ST_TRY(ensure_device(e));
    hipStream_t st = (hipStream_t)hip_stream;
    ST_TRY(settle(e, *s, true));
    ST_TRY(join(e, st));
    ST_TRY(defer_flush(*s, st));
    DevHeader h{};
    HIP_TRY(hipMemcpyAsync(&h, s->hdr, sizeof(h), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int k = h.k, ld = h.ld;
    if ((U && ldu < k) || (V && ldv < k)) return fail(ISVD_E_INVAL, "leading dimension below k = %d", k);
    auto pull = [&](const void* src, int64_t rows, double* dst, int64_t ldd) -> isvd_status {
        std::vector<char> buf((size_t)s->esz * round16(rows) * ld);
        HIP_TRY(hipMemcpyAsync(buf.data(), src, buf.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int64_t r = 0; r < rows; ++r)
            for (int c = 0; c < k; ++c)
                dst[r * ldd + c] = s->esz == 8 ? ((double*)buf.data())[uvo(r, c, ld)]
                                               : ((float*)buf.data())[uvo(r, c, ld)];
        return ISVD_OK;
    };
    if (U) ST_TRY(pull(s->U[h.cur], h.m, U, ldu));
    if (V) ST_TRY(pull(s->V[h.cur], h.n, V, ldv));
    if (S) {
        HIP_TRY(hipMemcpyAsync(S, s->S, sizeof(double) * k, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return ISVD_OK;
}

isvd_status isvd_get_matrix(isvd_engine* e, isvd_id id, double* A, int64_t lda, void* hip_stream) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    if (!A || lda < s->n) return fail(ISVD_E_INVAL, "null output or lda < n");
    ST_TRY(ensure_device(e));
    hipStream_t st = (hipStream_t)hip_stream;
    ST_TRY(settle(e, *s, true));
    ST_TRY(join(e, st));
    DevHeader h{};
    HIP_TRY(hipMemcpyAsync(&h, s->hdr, sizeof(h), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int64_t ldA = lda_of(s->cfg);
    std::vector<char> buf((size_t)s->esz * h.m * ldA);
    HIP_TRY(hipMemcpyAsync(buf.data(), s->A, buf.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t r = 0; r < h.m; ++r)
        for (int64_t c = 0; c < h.n; ++c)
            A[r * lda + c] = s->esz == 8 ? ((double*)buf.data())[r * ldA + c] : ((float*)buf.data())[r * ldA + c];
    return ISVD_OK;
}

isvd_status isvd_shape(isvd_engine* e, isvd_id id, int64_t* m, int64_t* n, int32_t* k) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    if (m) *m = s->m;
    if (n) *n = s->n;
    if (k) *k = s->k_target;
    return ISVD_OK;
}

}  // extern "C"

namespace {

// Move a released stream's block into the cache: an event on every engine
// stream (the reusing stream creation waits for them), then the block kept
// and the rest of the stream freed.  Its refresh, if any, has ended.
constexpr size_t kFreeBatch = 32;   // blocks past the cache's cap freed per device wait
isvd_status bcache_keep(isvd_engine* e, Stream* s) {
    if (e->bcache_bytes + s->base_bytes > e->bcache_cap) {
        // past the cap: free it with the next few, after one wait for the device
        e->to_free.push_back(s->base);
        e->used -= s->L.total;
        s->base = nullptr;
        free_stream(e, s);
        if (e->to_free.size() >= kFreeBatch) {
            (void)hipDeviceSynchronize();
            for (char* p : e->to_free) (void)hipFree(p);
            e->to_free.clear();
        }
        return ISVD_OK;
    }
    const std::vector<hipStream_t> es = engine_streams(e);
    while (e->ev_rel.size() < es.size()) {
        hipEvent_t ev;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        e->ev_rel.push_back(ev);
    }
    for (size_t q = 0; q < es.size(); ++q) HIP_TRY(hipEventRecord(e->ev_rel[q], es[q]));
    e->bcache.emplace(s->base_bytes, s->base);
    e->bcache_bytes += s->base_bytes;
    e->used -= s->L.total;
    s->base = nullptr;
    free_stream(e, s);
    return ISVD_OK;
}

// Released streams whose refresh has ended since: into the cache.
isvd_status release_poll(isvd_engine* e) {
    for (size_t q = 0; q < e->releasing.size();) {
        Stream* s = e->releasing[q];
        if (hipEventQuery(s->ev_ready) != hipSuccess) {
            ++q;
            continue;
        }
        e->releasing[q] = e->releasing.back();
        e->releasing.pop_back();
        s->refreshing = false;
        ST_TRY(bcache_keep(e, s));
    }
    return ISVD_OK;
}

}  // namespace

extern "C" {

isvd_status isvd_release(isvd_engine* e, isvd_id id) {
    Stream* s = nullptr;
    ST_TRY(get_stream(e, id, &s));
    (void)hipSetDevice(e->device);
    if (e->bcache_cap > 0 && s->base && !s->wbuf && !s->a_host) {
        ST_TRY(release_poll(e));
        // a refresh still running keeps the stream (its header slot and
        // block) until it ends; no wait here
        if (s->refreshing && hipEventQuery(s->ev_ready) != hipSuccess) {
            s->live = false;
            e->releasing.push_back(s);
            return ISVD_OK;
        }
        s->refreshing = false;
        return bcache_keep(e, s);
    }
    (void)hipDeviceSynchronize();
    e->rot_pending = false;
    free_stream(e, s);
    return ISVD_OK;
}

isvd_status isvd_tick(isvd_engine* e, int32_t count, const isvd_request* reqs, void* hip_stream) {
    if (!e || (count > 0 && !reqs)) return fail(ISVD_E_INVAL, "null engine or requests");
    if (count <= 0) return ISVD_OK;
    std::vector<Stream*> ss(count);
    if (e->seen_stamp.size() < e->streams.size()) e->seen_stamp.resize(e->streams.size(), 0);
    const uint64_t stamp = ++e->stamp;
    for (int q = 0; q < count; ++q) {
        const isvd_request& r = reqs[q];
        ST_TRY(get_stream(e, r.id, &ss[q]));
        Stream* s = ss[q];
        if (e->seen_stamp[r.id] == stamp) return fail(ISVD_E_INVAL, "stream %lld appears twice in one tick", (long long)r.id);
        e->seen_stamp[r.id] = stamp;
        if (r.kind == ISVD_ROW) {
            if (r.len != s->n) return fail(ISVD_E_SHAPE, "request %d: row length %lld != n %lld", q, (long long)r.len, (long long)s->n);
            if (s->m >= s->cfg.m_cap) return fail(ISVD_E_CAPACITY, "request %d: row capacity reached", q);
        } else if (r.kind == ISVD_COL) {
            if (r.len != s->m) return fail(ISVD_E_SHAPE, "request %d: column length %lld != m %lld", q, (long long)r.len, (long long)s->m);
            if (s->n >= s->cfg.n_cap) return fail(ISVD_E_CAPACITY, "request %d: column capacity reached", q);
        } else if (r.kind == ISVD_ENTRY) {
            if (r.i < 0 || r.i >= s->m || r.j < 0 || r.j >= s->n) return fail(ISVD_E_RANGE, "request %d: entry out of range", q);
            if (!std::isfinite(r.delta)) return fail(ISVD_E_NONFINITE, "request %d: delta not finite", q);
        } else {
            return fail(ISVD_E_INVAL, "request %d: bad kind %d", q, r.kind);
        }
        if (r.kind != ISVD_ENTRY) {
            if (!r.payload) return fail(ISVD_E_INVAL, "request %d: null payload", q);
            if ((r.dtype == ISVD_DTYPE_F64) != (s->esz == 8)) return fail(ISVD_E_INVAL, "request %d: payload dtype differs from storage", q);
        }
    }
    ST_TRY(ensure_device(e));
    hipStream_t st = (hipStream_t)hip_stream;
    // streams whose refresh still runs on a lane: the tick waits for those only
    for (int q = 0; q < count; ++q) {
        ST_TRY(settle(e, *ss[q], false));
        if (ss[q]->refreshing) HIP_TRY(hipStreamWaitEvent(st, ss[q]->ev_ready, 0));
    }
    // row appends of streams without a refresh policy pipeline with the
    // next tick; anything that reads U (column appends, entry updates,
    // trackers) waits for the pending U rotations, and a policy may refresh
    bool reads_u = false, pipelined = true;
    for (int q = 0; q < count; ++q) {
        if (reqs[q].kind != ISVD_ROW || ss[q]->angle) reads_u = true;
        if (reqs[q].kind != ISVD_ROW || ss[q]->cfg.policy.kind != ISVD_POL_NONE) pipelined = false;
    }
    pipelined = pipelined && e->pipelining;
    if (reads_u) ST_TRY(join(e, st));
    for (int q = 0; q < count; ++q)
        if (reqs[q].kind != ISVD_ROW) ST_TRY(defer_flush(*ss[q], st));
    std::map<std::pair<int, int>, int> gi;   // (storage size + BF16 flag, bucket)
    std::vector<Group> groups;
    for (int q = 0; q < count; ++q) {
        Stream& s = *ss[q];
        auto key = std::make_pair(s.esz * 2 + (s.bf16 ? 1 : 0), s.kc);
        if (!gi.count(key)) {
            gi[key] = (int)groups.size();
            groups.emplace_back();
            groups.back().fp64 = s.esz == 8;
            groups.back().bf16 = s.bf16;
            groups.back().kc = s.kc;
            groups.back().rows = rows_for(e, s.kc, s.esz == 8);
            groups.back().var = var_for(e, s.kc, s.esz == 8);
        }
        Group& g = groups[gi[key]];
        const isvd_request& r = reqs[q];
        Req rq = make_req(e, s, r.kind, r.payload, r.i, r.j, r.delta, k_keep_for(s, r.kind));
        g.all.push_back(rq);
        if (r.kind != ISVD_ENTRY) g.proj.push_back(rq);
        g.ids.push_back(r.id);
        g.rotU_cap += (int)cdiv(s.cfg.m_cap, g.rows);
    }
    // deferred-U ticks of row appends without policies replay a captured graph
    bool graph = e->tick_graphs && e->defer_u && !e->profiling;
    for (int q = 0; q < count && graph; ++q)
        graph = reqs[q].kind == ISVD_ROW && ss[q]->cfg.policy.kind == ISVD_POL_NONE && !ss[q]->angle &&
                !ss[q]->refreshing;
    if (graph)
        ST_TRY(run_groups_graph(e, groups, st, pipelined));
    else
        ST_TRY(run_groups(e, groups, st, pipelined));
    std::vector<Track> tracks;
    std::vector<char> tfp;
    for (int q = 0; q < count; ++q)
        if (ss[q]->angle) {
            tracks.push_back(make_track(*ss[q], reqs[q].kind, reqs[q].payload));
            tfp.push_back(ss[q]->esz == 8);
        }
    ST_TRY(run_tracks(e, tracks, tfp, st));
    for (int q = 0; q < count; ++q) {
        Stream& s = *ss[q];
        if (reqs[q].kind == ISVD_ROW) s.m += 1;
        if (reqs[q].kind == ISVD_COL) s.n += 1;
        s.t += 1;
    }
    // trackers of the streams whose policy reads them: one copy of the header array
    int nh = 0;
    for (int q = 0; q < count; ++q) nh += policy_needs_header(*ss[q]) ? 1 : 0;
    if (nh > 0) {
        HIP_TRY(hipMemcpyAsync(e->hdr_mirror, e->hdr_dev, sizeof(DevHeader) * e->hdr_hi, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    Deferred d;
    for (int q = 0; q < count; ++q)
        ST_TRY(after_update(e, *ss[q], st, policy_needs_header(*ss[q]) ? e->hdr_mirror + ss[q]->slot : nullptr, &d));
    for (size_t i0 = 0; i0 < d.shrink.size(); i0 += kShrinkBatch) {
        ShrinkList L{};
        L.n = (int)std::min<size_t>(kShrinkBatch, d.shrink.size() - i0);
        for (int i = 0; i < L.n; ++i) {
            L.hdr[i] = d.shrink[i0 + i]->hdr;
            L.S[i] = d.shrink[i0 + i]->S;
        }
        k_shrink_many<<<1, kShrinkBatch, 0, st>>>(L);
        HIP_TRY(hipGetLastError());
    }
    if (!d.checks.empty()) ST_TRY(check_batch(e, d.checks, st));
    if (!d.refresh.empty()) ST_TRY(refresh_batch(e, d.refresh, st));
    return ISVD_OK;
}

}  // extern "C"
