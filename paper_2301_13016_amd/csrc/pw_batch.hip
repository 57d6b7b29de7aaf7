// Batched form: many independent subdomains in one persistent launch.
//
// The paper scales by decomposing the grid into independent parts, each on
// its own compute unit (Sec. 5).  On one MI355X the analogue is a batch of
// MONC-rank-sized subdomains of different shapes served by a single
// persistent grid: the host flattens every subdomain's (strip, z-chunk) work
// items into one list (per-subdomain prefix offsets in a device descriptor
// table), and each wavefront of the persistent grid repeatedly takes the next
// item from a device counter, finds its subdomain by binary search over the
// prefix offsets, and runs the same strip march as the single-grid kernel.
// Items are numbered z-chunk fastest, then x, then y inside a subdomain, so
// wavefronts that start at about the same time work on neighbouring strips.
//
// The list is cut into 8 contiguous ranges, one per XCD, each with its own
// counter: workgroups are dispatched to the XCDs round robin, so a wavefront
// takes items from its own XCD's range first, and neighbouring strips -- which
// share y-halo rows -- run under one L2.  (With one global counter they were
// spread over all eight L2s and reads rose to 1.8x the algorithmic bytes.)
// When its range is exhausted a wavefront takes items from the other ranges
// in turn, which balances the tail.
//
// The counters are cleared by a small kernel launched just before the
// persistent kernel (a kernel node rather than a memset node, so the pair can
// be captured in a HIP graph and replayed).  A wavefront exits when every
// counter has passed the end of its range; each attempt either takes an item
// or moves to the next range, so every wavefront terminates.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "pw_stencil.h"

namespace pw {
namespace {

using namespace dev;

template <typename Tin> struct BatchSub {
    FwdK<Tin> k;
    int64_t first;   // index of the subdomain's first work item
    int32_t px;      // columns per lane of its strips
};

constexpr int kXcds = 8;         // XCDs of an MI355X
constexpr int kCtrStride = 16;   // counters 128 bytes apart

__global__ void batch_reset_kernel(unsigned long long *counter) {
    if (threadIdx.x < kXcds) counter[threadIdx.x * kCtrStride] = 0ull;
}

// Depth: planes in flight (1 or 2).  MaxT: workgroup size bound (built for
// 256 and 512 threads, as the single-grid kernels).  PX 0: each subdomain's
// strips have the width its work-list entry names (1 or 2 columns per lane;
// the choice is wave-uniform, made per work item).
template <typename Tin, int PX, int RY, int Depth, int MaxT>
__global__ __launch_bounds__(MaxT) void pw_batch_kernel(const BatchSub<Tin> *__restrict__ subs, int nsub,
                                                       int64_t nitems, unsigned long long *counter) {
    const int lane = threadIdx.x & 63;
    const int home = static_cast<int>(blockIdx.x) & (kXcds - 1);
    for (int r = 0; r < kXcds; ++r) {
      const int x = (home + r) & (kXcds - 1);
      const int64_t first = nitems * x / kXcds, last = nitems * (x + 1) / kXcds;
      for (;;) {
        unsigned long long got = 0ull;
        if (lane == 0) got = atomicAdd(counter + x * kCtrStride, 1ull);
        const int64_t item = first + static_cast<int64_t>(
            (static_cast<unsigned long long>(__builtin_amdgcn_readfirstlane(static_cast<unsigned>(got >> 32))) << 32) |
            static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<unsigned>(got))));
        if (item >= last) break;
        int lo = 0, hi = nsub - 1;   // last subdomain whose first item <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (subs[mid].first <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const FwdK<Tin> &a = subs[lo].k;
        const int64_t local = item - subs[lo].first;
        const int cz = static_cast<int>(local % a.nzc);
        const int64_t t2 = local / a.nzc;
        const int tx = static_cast<int>(t2 % a.ntx);
        const int ty = static_cast<int>(t2 / a.ntx);
        if constexpr (PX == 0) {
            if (subs[lo].px == 2)
                strip_march<Tin, 2, RY, Depth>(a, tx, ty, cz);
            else
                strip_march<Tin, 1, RY, Depth>(a, tx, ty, cz);
        } else {
            strip_march<Tin, PX, RY, Depth>(a, tx, ty, cz);
        }
      }
    }
}

using Tin = float;   // the batched form runs FP32 storage

template <int PX, int RY, int Depth, int MaxT> const void *kernel_ptr() {
    return reinterpret_cast<const void *>(&pw_batch_kernel<Tin, PX, RY, Depth, MaxT>);
}

template <int Depth, int MaxT> const void *batch_kernel_t(const TileCfg &c) {
    switch (c.px * 16 + c.ry) {
        case 0 + 1: return kernel_ptr<0, 1, Depth, MaxT>();
        case 0 + 2: return kernel_ptr<0, 2, Depth, MaxT>();
        case 0 + 4: return kernel_ptr<0, 4, Depth, MaxT>();
        case 16 + 1: return kernel_ptr<1, 1, Depth, MaxT>();
        case 16 + 2: return kernel_ptr<1, 2, Depth, MaxT>();
        case 16 + 4: return kernel_ptr<1, 4, Depth, MaxT>();
        case 32 + 1: return kernel_ptr<2, 1, Depth, MaxT>();
        case 32 + 2: return kernel_ptr<2, 2, Depth, MaxT>();
        case 32 + 4: return kernel_ptr<2, 4, Depth, MaxT>();
        case 64 + 1: return kernel_ptr<4, 1, Depth, MaxT>();
        case 64 + 2: return kernel_ptr<4, 2, Depth, MaxT>();
    }
    return nullptr;
}

// The instantiation a tile runs (nullptr: none).
const void *batch_kernel(const TileCfg &c) {
    if (c.share != 0) return nullptr;   // independent wavefronts only
    if (c.depth == 2) return c.wpb <= 4 ? batch_kernel_t<2, 256>(c) : batch_kernel_t<2, 512>(c);
    if (c.depth == 1) return c.wpb <= 4 ? batch_kernel_t<1, 256>(c) : batch_kernel_t<1, 512>(c);
    return nullptr;
}

hipError_t launch_batch(const TileCfg &c, dim3 g, dim3 b, hipStream_t s, const BatchSub<Tin> *d, int n,
                        int64_t items, unsigned long long *ctr) {
    // every instantiation has the same signature: launch through its pointer
    const void *k = batch_kernel(c);
    if (!k) return hipErrorInvalidDeviceFunction;
    void *args[] = {&d, &n, &items, &ctr};
    return hipLaunchKernel(k, g, b, args, 0, s);
}

TileCfg default_batch_tile() {
    TileCfg c;
    c.px = 1;
    c.ry = 2;
    c.zlen = 64;
    c.wpb = 4;
    return c;
}

}  // namespace
}  // namespace pw

using namespace pw;

struct pw_batch {
    std::vector<FwdArgs> subs;
    pw_dtype dtype = PW_F32;
    TileCfg tile;
    int device = 0;
    int cus = 256;
    BatchSub<Tin> *d_table = nullptr;
    unsigned long long *d_counter = nullptr;
    int64_t nitems = 0;
    int blocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void drop_graph(pw_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Columns per lane of a subdomain nx wide under the per-subdomain choice:
// 2 where that leaves no more lanes idle than 1 (fewer, wider vector loads
// per point), else 1 (e.g. 33..64 or 129..192 columns: half a 128-column
// strip would be empty).
int sub_columns(int64_t nx) {
    const int64_t s1 = (nx + 63) / 64 * 64, s2 = (nx + 127) / 128 * 128;
    return s2 == s1 ? 2 : 1;
}

// Builds and uploads the work list for `tile` (synchronous upload).
pw_status build_table(pw_batch *b, const TileCfg &tile) {
    std::vector<BatchSub<Tin>> h(b->subs.size());
    int64_t first = 0;
    for (size_t i = 0; i < b->subs.size(); ++i) {
        const FwdArgs &g = b->subs[i];
        FwdK<Tin> &a = h[i].k;
        a.u = static_cast<const Tin *>(g.u);
        a.v = static_cast<const Tin *>(g.v);
        a.w = static_cast<const Tin *>(g.w);
        a.su = static_cast<float *>(g.su);
        a.sv = static_cast<float *>(g.sv);
        a.sw = static_cast<float *>(g.sw);
        a.tzc1 = static_cast<const float *>(g.tzc1);
        a.tzc2 = static_cast<const float *>(g.tzc2);
        a.tzd1 = static_cast<const float *>(g.tzd1);
        a.tzd2 = static_cast<const float *>(g.tzd2);
        a.tcx = static_cast<float>(g.tcx);
        a.tcy = static_cast<float>(g.tcy);
        a.nx = static_cast<int32_t>(g.nx);
        a.ny = static_cast<int32_t>(g.ny);
        a.nz = static_cast<int32_t>(g.nz);
        a.h = g.h;
        a.in_sz = g.in_sz;
        a.out_sz = g.out_sz;
        a.in_sy = static_cast<int32_t>(g.in_sy);
        a.out_sy = static_cast<int32_t>(g.out_sy);
        const int px = tile.px > 0 ? tile.px : sub_columns(g.nx);
        h[i].px = px;
        a.ntx = static_cast<int32_t>((g.nx + 64 * px - 1) / (64 * px));
        a.nty = static_cast<int32_t>((g.ny + tile.ry - 1) / tile.ry);
        // split nz evenly into chunks of at most tile.zlen levels
        const int64_t chunks = (g.nz + tile.zlen - 1) / tile.zlen;
        a.zlen = static_cast<int32_t>((g.nz + chunks - 1) / chunks);
        a.nzc = static_cast<int32_t>((g.nz + a.zlen - 1) / a.zlen);
        a.wpb = 1;
        h[i].first = first;
        first += static_cast<int64_t>(a.ntx) * a.nty * a.nzc;
    }
    BatchSub<Tin> *d = nullptr;
    const size_t bytes = h.size() * sizeof(BatchSub<Tin>);
    if (hipMalloc(&d, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PW_ERR_ALLOC, "work list allocation failed");
    }
    hipError_t e = hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "work list upload");
    }
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel(tile), 64 * tile.wpb, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    if (b->d_table) (void)hipFree(b->d_table);
    b->d_table = d;
    b->nitems = first;
    b->tile = tile;
    int64_t blocks = static_cast<int64_t>(per_cu) * b->cus;
    const int64_t max_useful = (first + tile.wpb - 1) / tile.wpb;   // one item per wavefront at least
    if (blocks > max_useful) blocks = max_useful;
    if (blocks < 1) blocks = 1;
    b->blocks = static_cast<int>(blocks);
    drop_graph(b);
    return PW_OK;
}

pw_status enqueue(pw_batch *b, hipStream_t s) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, b->d_counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "counter reset launch");
    e = launch_batch(b->tile, dim3(static_cast<unsigned>(b->blocks)), dim3(64 * b->tile.wpb), s, b->d_table,
                     static_cast<int>(b->subs.size()), b->nitems, b->d_counter);
    if (e == hipSuccess) e = hipGetLastError();
    return hip_fail(e, "batched kernel launch");
}

bool batch_tile_ok(const TileCfg &c) {
    if (c.zlen < 1 || c.share != 0) return false;
    if (c.px == 0) {
        TileCfg c1 = c, c2 = c;
        c1.px = 1;
        c2.px = 2;
        return tile_supported(c1, PW_F32) && tile_supported(c2, PW_F32) && batch_kernel(c) != nullptr;
    }
    return tile_supported(c, PW_F32) && batch_kernel(c) != nullptr;
}

}  // namespace

extern "C" {

pw_status pw_batch_create(const pw_batch_item *items, int32_t n, pw_dtype dtype, const pw_tile *tile,
                          pw_batch **out) {
    if (!out) return fail(PW_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!items || n < 1) return fail(PW_ERR_INVALID_ARG, "need at least one item");
    if (n > (1 << 20)) return fail(PW_ERR_INVALID_ARG, "too many items");
    if (dtype != PW_F32) return fail(PW_ERR_UNSUPPORTED, "the batched form supports PW_F32 storage");
    TileCfg cfg = default_batch_tile();
    if (tile) {
        cfg = TileCfg{tile->cols_per_lane, tile->rows_per_strip, tile->zlen, tile->waves_per_group,
                      tile->prefetch == 0 ? 1 : tile->prefetch, tile->share_rows};
        if (!batch_tile_ok(cfg))
            return fail(PW_ERR_INVALID_ARG,
                        "unsupported batch tile cols=%d rows=%d zlen=%d waves=%d prefetch=%d share_rows=%d", cfg.px,
                        cfg.ry, cfg.zlen, cfg.wpb, tile->prefetch, tile->share_rows);
    }
    std::vector<FwdArgs> subs(static_cast<size_t>(n));
    for (int32_t i = 0; i < n; ++i) {
        const pw_batch_item &it = items[i];
        const pw_layout *L = &it.layout;
        if (!it.layout.in_sy && !it.layout.in_sz && !it.layout.out_sy && !it.layout.out_sz) L = nullptr;
        pw_status st = validate_forward(&it.grid, L, dtype, it.u, it.v, it.w, &it.coeffs, it.su, it.sv, it.sw, &subs[i]);
        if (st != PW_OK) {
            char msg[512];
            std::snprintf(msg, sizeof msg, "%s", pw_last_error());
            return fail(st, "item %d: %s", i, msg);
        }
    }
    // No output may overlap any other array of any item (inputs and
    // coefficients may share memory: they are only read; the coefficients
    // are read through the scalar cache).  One sort and sweep: in lo order, a
    // range overlaps an earlier one iff it starts below the largest earlier
    // end, so it suffices to track that end over all ranges and over outputs.
    struct Span {
        uintptr_t lo, hi;
        int32_t item;
        bool out;
    };
    std::vector<Span> spans;
    spans.reserve(static_cast<size_t>(n) * 10);
    for (int32_t i = 0; i < n; ++i) {
        uintptr_t ri[3][2], ro[3][2];
        forward_ranges(subs[i], ri, ro);
        for (int f = 0; f < 3; ++f) {
            spans.push_back(Span{ri[f][0], ri[f][1], i, false});
            spans.push_back(Span{ro[f][0], ro[f][1], i, true});
        }
        const void *cp[4] = {items[i].coeffs.tzc1, items[i].coeffs.tzc2, items[i].coeffs.tzd1, items[i].coeffs.tzd2};
        for (const void *c : cp) {
            const uintptr_t lo = reinterpret_cast<uintptr_t>(c);
            spans.push_back(Span{lo, lo + uintptr_t(items[i].grid.nz) * sizeof(float), i, false});
        }
    }
    std::sort(spans.begin(), spans.end(), [](const Span &a, const Span &b) { return a.lo < b.lo; });
    uintptr_t end_all = 0, end_out = 0;
    int32_t who_all = -1, who_out = -1;
    for (const Span &s : spans) {
        if (s.hi <= s.lo) continue;
        if (s.out && s.lo < end_all)
            return fail(PW_ERR_INVALID_ARG, "an output of item %d overlaps an array of item %d", s.item, who_all);
        if (!s.out && s.lo < end_out)
            return fail(PW_ERR_INVALID_ARG, "an output of item %d overlaps an array of item %d", who_out, s.item);
        if (s.hi > end_all) {
            end_all = s.hi;
            who_all = s.item;
        }
        if (s.out && s.hi > end_out) {
            end_out = s.hi;
            who_out = s.item;
        }
    }
    for (int32_t i = 0; i < n; ++i) {
        pw_status st = check_forward_on_device(subs[i]);
        if (st != PW_OK) {
            char msg[512];
            std::snprintf(msg, sizeof msg, "%s", pw_last_error());
            return fail(st, "item %d: %s", i, msg);
        }
    }
    pw_batch *b = new (std::nothrow) pw_batch;
    if (!b) return fail(PW_ERR_ALLOC, "host allocation failed");
    b->subs.swap(subs);
    b->dtype = dtype;
    (void)hipGetDevice(&b->device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess && prop.multiProcessorCount > 0)
        b->cus = prop.multiProcessorCount;
    if (hipMalloc(&b->d_counter, kXcds * kCtrStride * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return fail(PW_ERR_ALLOC, "counter allocation failed");
    }
    pw_status st = build_table(b, cfg);
    if (st != PW_OK) {
        pw_batch_destroy(b);
        return st;
    }
    *out = b;
    return PW_OK;
}

pw_status pw_batch_run(pw_batch *b, void *hip_stream) {
    if (!b) return fail(PW_ERR_INVALID_ARG, "batch is NULL");
    return enqueue(b, static_cast<hipStream_t>(hip_stream));
}

pw_status pw_batch_capture(pw_batch *b, void *hip_stream) {
    if (!b) return fail(PW_ERR_INVALID_ARG, "batch is NULL");
    if (!hip_stream) return fail(PW_ERR_INVALID_ARG, "graph capture needs a non-NULL stream");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    pw_status st = enqueue(b, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (st != PW_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    b->graph = g;
    b->exec = x;
    return PW_OK;
}

pw_status pw_batch_replay(pw_batch *b, void *hip_stream) {
    if (!b) return fail(PW_ERR_INVALID_ARG, "batch is NULL");
    if (!b->exec) return fail(PW_ERR_INVALID_ARG, "batch has no captured graph (pw_batch_capture)");
    return hip_fail(hipGraphLaunch(b->exec, static_cast<hipStream_t>(hip_stream)), "hipGraphLaunch");
}

pw_status pw_batch_tune(pw_batch *b, void *hip_stream, pw_tile *chosen) {
    if (!b) return fail(PW_ERR_INVALID_ARG, "batch is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return hip_fail(hipGetLastError(), "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(hipGetLastError(), "hipEventCreate");
    }
    // mean ms of `reps` runs of the batch under tile c, after one warm-up run
    auto time_tile = [&](const TileCfg &c, int reps, float *ms) -> pw_status {
        pw_status st = build_table(b, c);
        if (st == PW_OK) st = enqueue(b, s);
        if (st != PW_OK) return st;
        if (hipEventRecord(e0, s) != hipSuccess) return hip_fail(hipGetLastError(), "hipEventRecord");
        for (int r = 0; r < reps && st == PW_OK; ++r) st = enqueue(b, s);
        if (st != PW_OK) return st;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return hip_fail(hipGetLastError(), "timing");
        *ms /= reps;
        return PW_OK;
    };
    const TileCfg start = b->tile;
    TileCfg best = start;
    std::vector<std::pair<float, TileCfg>> t;
    pw_status st = PW_OK;
    for (int px : {0, 1, 2, 4})
        for (int ry : {1, 2, 4})
            for (int zl : {32, 64, 128, 256})
                for (int wpb : {1, 4})
                    for (int depth : {1, 2}) {
                            if (st != PW_OK) break;
                            TileCfg c;
                            c.px = px;
                            c.ry = ry;
                            c.zlen = zl;
                            c.wpb = wpb;
                            c.depth = depth;
                            if (!batch_tile_ok(c)) continue;
                            float ms = -1.f;
                            st = time_tile(c, 3, &ms);
                            if (st == PW_OK && ms > 0.f) t.emplace_back(ms, c);
                        }
    // the three fastest again over more runs (less sensitive to noise)
    if (st == PW_OK && !t.empty()) {
        std::sort(t.begin(), t.end(), [](const std::pair<float, TileCfg> &x, const std::pair<float, TileCfg> &y) {
            return x.first < y.first;
        });
        float best_ms = -1.f;
        for (size_t r = 0; r < t.size() && r < 3 && st == PW_OK; ++r) {
            float ms = -1.f;
            st = time_tile(t[r].second, 10, &ms);
            if (st == PW_OK && ms > 0.f && (best_ms < 0.f || ms < best_ms)) {
                best_ms = ms;
                best = t[r].second;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const pw_status st2 = build_table(b, st == PW_OK ? best : start);
    if (st != PW_OK) return st;
    if (st2 != PW_OK) return st2;
    if (chosen) *chosen = to_tile(best);
    return PW_OK;
}

pw_status pw_batch_info(const pw_batch *b, pw_tile *tile, int64_t *work_items, int32_t *workgroups) {
    if (!b) return fail(PW_ERR_INVALID_ARG, "batch is NULL");
    if (tile) *tile = to_tile(b->tile);
    if (work_items) *work_items = b->nitems;
    if (workgroups) *workgroups = b->blocks;
    return PW_OK;
}

pw_status pw_batch_destroy(pw_batch *b) {
    if (!b) return PW_OK;
    drop_graph(b);
    if (b->d_table) (void)hipFree(b->d_table);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
    return PW_OK;
}

}  // extern "C"
