// C ABI of the library (declared in include/ata.h): argument validation,
// plan cache, workspace, and the launch sequence of one Gram product.
#include "ata.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <tuple>
#include <vector>

#include "launch.hpp"
#include "plan.hpp"

using namespace ata;

namespace {

struct PlanKey {
    int32_t mode;
    int64_t m, n, lda, b;
    int32_t depth;
    bool fb;
    int32_t tile_cfg;
    int64_t split;
    bool fuse;
    int32_t variant;
    int64_t slots;
    bool bounded;
    bool overlap;
    bool fuse_combine = false;
    bool operator<(const PlanKey& o) const {
        return std::tie(mode, m, n, lda, b, depth, fb, tile_cfg, split, fuse, variant, slots, bounded, overlap,
                        fuse_combine) <
               std::tie(o.mode, o.m, o.n, o.lda, o.b, o.depth, o.fb, o.tile_cfg, o.split, o.fuse, o.variant,
                        o.slots, o.bounded, o.overlap, o.fuse_combine);
    }
};

// A plan plus its descriptor arrays resident in device memory.
struct DevicePlan {
    Plan plan;
    void* d_buf = nullptr;
    LeafDesc* d_leaves = nullptr;
    LeafDesc* d_fb_leaves = nullptr;
    std::vector<PresumDesc*> d_presum;
    PackDesc* d_pack = nullptr;
    Pack8Desc* d_pack8 = nullptr;
    std::vector<CombineDesc*> d_combine;
    NodeDesc* d_nodes = nullptr;
    ColDesc* d_col1 = nullptr;
    ColDesc* d_col2 = nullptr;
    ReduceDesc* d_reduce = nullptr;
    std::vector<Sum2Desc*> d_sums;
    std::vector<AccumDesc*> d_accum;
    // bounded workspace: the stages after this one (this plan is stage 0),
    // and the largest stage's arena
    std::vector<std::unique_ptr<DevicePlan>> stages;
    int64_t stage_arena_elems = 0;
    ~DevicePlan() { if (d_buf) (void)hipFree(d_buf); }
    int64_t arena_elems() const { return stages.empty() ? plan.arena_elems : stage_arena_elems; }
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Autotune table key: dtype and half-octave buckets of m and n.
struct TuneKey {
    int32_t mode;
    int32_t mb, nb;
    bool operator<(const TuneKey& o) const { return std::tie(mode, mb, nb) < std::tie(o.mode, o.mb, o.nb); }
};

int32_t bucket(int64_t x) { return x <= 1 ? 0 : (int32_t)std::lround(2.0 * std::log2((double)x)); }

struct BatchKey {
    int32_t mode;
    int64_t b;
    int32_t depth;
    bool fb;
    int32_t tile_cfg;
    int64_t split;
    bool fuse;
    int32_t variant;
    int64_t slots;
    std::vector<int64_t> shapes;   // m, n, lda per problem
    bool operator<(const BatchKey& o) const {
        return std::tie(mode, b, depth, fb, tile_cfg, split, fuse, variant, slots, shapes) <
               std::tie(o.mode, o.b, o.depth, o.fb, o.tile_cfg, o.split, o.fuse, o.variant, o.slots, o.shapes);
    }
};

// Plan-cache key of a general product C = A^T B.
struct GemmKey {
    int32_t mode;
    int64_t m, n, k, lda, ldb, ldc, b;
    int32_t depth, tile_cfg;
    int64_t split;
    bool fuse;
    int32_t variant;
    int64_t slots;
    bool fuse_combine = false;
    bool operator<(const GemmKey& o) const {
        return std::tie(mode, m, n, k, lda, ldb, ldc, b, depth, tile_cfg, split, fuse, variant, slots, fuse_combine) <
               std::tie(o.mode, o.m, o.n, o.k, o.lda, o.ldb, o.ldc, o.b, o.depth, o.tile_cfg, o.split, o.fuse,
                        o.variant, o.slots, o.fuse_combine);
    }
};

std::vector<int64_t> batch_signature(int32_t mode, int64_t batch, const int64_t* m, const int64_t* n,
                                     const int64_t* lda) {
    std::vector<int64_t> sig;
    sig.reserve(1 + 3 * (size_t)batch);
    sig.push_back(mode);
    for (int64_t i = 0; i < batch; ++i) {
        sig.push_back(m[i]);
        sig.push_back(n[i]);
        sig.push_back(lda[i]);
    }
    return sig;
}

// A merged batch plan with its own device buffers and captured graph.
struct BatchEntry {
    std::unique_ptr<DevicePlan> dp;
    std::vector<ColDesc> col1, col2;
    ColDesc* d_col1 = nullptr;
    ColDesc* d_col2 = nullptr;
    void* aux = nullptr;               // ptr arrays | counter | flags | partials | nu
    size_t aux_bytes = 0;
    const void** d_A = nullptr;
    void** d_C = nullptr;
    unsigned long long* d_counter = nullptr;
    bool graph_persistent = false;     // leaf launch form the graph was captured with
    uint8_t* d_flags = nullptr;
    double* d_partial = nullptr;
    double* d_nu = nullptr;
    void** pinned = nullptr;           // A pointers then C pointers (page-locked)
    int64_t nprob = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t arena_gen = 0;            // arena generation the graph was captured with
    hipEvent_t done = nullptr;
    bool launched = false;
    ~BatchEntry() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (done) (void)hipEventDestroy(done);
        if (pinned) (void)hipHostFree(pinned);
        if (aux) (void)hipFree(aux);
    }
};

// A plan of ata_gram_noalloc: descriptors, arena and auxiliary block laid
// out in the device's static workspace, the descriptor blob on the host.
struct StaticPlan {
    DevicePlan dp;                     // d_buf stays null: nothing is owned
    std::vector<unsigned char> blob;   // descriptor bytes, copied in by every call
    size_t arena_off = 0, aux_off = 0, total = 0;
};

// The static workspace of ata_gram_noalloc.  Host code never uses this name
// as an address (on the host it is only a stand-in for the symbol): each
// device's address comes from hipGetSymbolAddress at the first ata_create on
// that device and is kept in scratch_base.
static __device__ __align__(256) unsigned char scratch[ATA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
unsigned char* scratch_base[kMaxDevices] = {};

// This device's address of the static workspace (looked up once; the caller
// has made the device current).
ata_status_t scratch_address(int dev, unsigned char*& out) {
    out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return ATA_ERR_NOT_SUPPORTED;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_base[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return ATA_ERR_HIP;
        scratch_base[dev] = static_cast<unsigned char*>(ptr);
    }
    out = scratch_base[dev];
    return ATA_OK;
}

}  // namespace

struct ata_ctx {
    int device = 0;
    PlanOptions popt;
    bool residual = false;
    uint64_t seed = 0x5EEDull;
    int64_t ws_limit = 0;
    int chunk = 16;                    // leaf tiles per XCD per window
    int band = 4;                      // GEMM leaf tile rows per band
    int64_t split_target = 2048;       // split-K below this many tiles per leaf launch (0: never)
    std::map<PlanKey, std::unique_ptr<DevicePlan>> plans;
    void* arena = nullptr;
    size_t arena_cap = 0;
    void* aux = nullptr;       // flags | column-norm partials | nu | residual work | residual
    size_t aux_cap = 0;
    hipStream_t last_stream = nullptr;
    bool pending_flags = false, pending_residual = false;
    uint8_t* last_flags = nullptr;
    double* last_residual = nullptr;
    int64_t last_nodes = 0;
    ata_report_t report{};
    // autotuned choices and the device architecture they were measured on
    std::map<TuneKey, ata_tune_entry_t> tune;
    std::string arch;
    // batches: merged plans, captured graphs, internal capture stream
    std::map<BatchKey, std::unique_ptr<BatchEntry>> batches;
    std::map<GemmKey, std::unique_ptr<DevicePlan>> gemm_plans;
    // column equilibration: option, norm tasks per (m, n, lda), buffers
    bool equilibrate = false;
    std::map<std::tuple<int64_t, int64_t, int64_t>, std::unique_ptr<DevicePlan>> eq_plans;
    void* eq = nullptr;
    size_t eq_cap = 0;
    // staging for the BLAS-style conveniences (a scaled product's result, a
    // transposed input)
    void* tmp = nullptr;
    size_t tmp_cap = 0;
    // batch autotuning: one (cutoff, depth, tile) per batch signature (dtype,
    // then m, n, lda of every member); per-shape table entries apply inside
    // batches only when batch_use_table is set
    std::map<std::vector<int64_t>, ata_tune_entry_t> batch_tune;
    bool batch_use_table = false;
    hipStream_t batch_stream = nullptr;
    hipEvent_t batch_in = nullptr;
    bool batch_graph = true;
    int batch_persistent = -1;         // 0 grid, 1 persistent, -1 automatic
    int leaf_persistent = -1;
    bool balance_tail = true;          // split the leaves of an underfilled last round
    bool bounded = false;              // Strassen roots product by product (make_staged_plan)
    int overlap = 0;                   // pre-sums beside the A-only leaves: 1 on, 0 off, -1 automatic (off)
    hipStream_t side = nullptr;        // second stream of an overlapped call (default priority)
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    uint64_t arena_gen = 0;
    // phase profiling: six events per profiled call, summed at report time
    bool profile = false;
    std::vector<hipEvent_t> events;   // pool, grows on demand
    size_t events_used = 0;
    int64_t profiled_calls = 0;
    double phase_ms[5] = {0, 0, 0, 0, 0};
    // set once a call has been enqueued on a capturing stream: from then on
    // superseded workspace buffers are retired, not freed (see ensure)
    bool captured = false;
    std::vector<void*> retired;
    // column norms and spread flags of the last ata_gram call with the
    // spread check (ata_get_spread); null plan when there is none
    const DevicePlan* spread_plan = nullptr;
    const double* spread_nu = nullptr;
    const uint8_t* spread_flags = nullptr;
    hipStream_t spread_stream = nullptr;
    // ata_gram_noalloc: this device's static workspace and the plans laid out
    // in it (descriptor blobs kept on the host, copied in by every call)
    unsigned char* scratch = nullptr;
    std::map<PlanKey, std::unique_ptr<StaticPlan>> static_plans;
};

namespace {

ata_status_t hip_status(hipError_t e) { return e == hipSuccess ? ATA_OK : ATA_ERR_HIP; }

// Remember that work of this handle is being recorded into a graph.
void note_capture(ata_ctx* h, void* stream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(static_cast<hipStream_t>(stream), &cs) == hipSuccess &&
        cs != hipStreamCaptureStatusNone)
        h->captured = true;
}

constexpr int EVENTS_PER_CALL = 6;

// Sum the elapsed times of all recorded calls (waits for them) and reset.
hipError_t drain_events(ata_ctx* h) {
    for (size_t base = 0; base + EVENTS_PER_CALL <= h->events_used; base += EVENTS_PER_CALL) {
        hipError_t e = hipEventSynchronize(h->events[base + EVENTS_PER_CALL - 1]);
        if (e != hipSuccess) return e;
        for (int ph = 0; ph < 5; ++ph) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, h->events[base + ph], h->events[base + ph + 1]);
            if (e != hipSuccess) return e;
            h->phase_ms[ph] += ms;
        }
        ++h->profiled_calls;
    }
    h->events_used = 0;
    return hipSuccess;
}

void clear_events(ata_ctx* h) {
    for (hipEvent_t ev : h->events) (void)hipEventDestroy(ev);
    h->events.clear();
    h->events_used = 0;
}

// Grow one of the handle's device buffers.  A smaller buffer is freed
// (hipFree waits for outstanding work on the device) unless a call on this
// handle has been recorded into a caller's graph: that graph still holds the
// old address, so the buffer is kept until ata_destroy.
ata_status_t ensure(ata_ctx* h, void*& ptr, size_t& cap, size_t bytes) {
    if (bytes <= cap) return ATA_OK;
    if (ptr) {
        if (h && h->captured) {
            h->retired.push_back(ptr);
        } else if (hipFree(ptr) != hipSuccess) {
            return ATA_ERR_HIP;
        }
        ptr = nullptr;
        cap = 0;
    }
    if (hipMalloc(&ptr, bytes) != hipSuccess) {
        ptr = nullptr;
        return ATA_ERR_OUT_OF_MEMORY;
    }
    cap = bytes;
    return ATA_OK;
}

// Lay the plan's descriptor arrays out in one blob (each array 256-byte
// aligned) and point the DevicePlan's device arrays at `base` plus their
// offsets.  The blob goes to `host`; returns its size in bytes.
size_t layout_descriptors(DevicePlan& dp, unsigned char* base, std::vector<unsigned char>& host) {
    const Plan& p = dp.plan;
    size_t bytes = align256(p.leaves.size() * sizeof(LeafDesc));
    for (auto& l : p.presum) bytes += align256(l.size() * sizeof(PresumDesc));
    for (auto& l : p.combine) bytes += align256(l.size() * sizeof(CombineDesc));
    bytes += align256(p.nodes.size() * sizeof(NodeDesc));
    bytes += align256(p.pack.size() * sizeof(PackDesc));
    bytes += align256(p.fb_leaves.size() * sizeof(LeafDesc));
    bytes += align256(p.pack8.size() * sizeof(Pack8Desc));
    bytes += align256(p.col1.size() * sizeof(ColDesc));
    bytes += align256(p.col2.size() * sizeof(ColDesc));
    bytes += align256(p.reduce.size() * sizeof(ReduceDesc));
    for (auto& l : p.sums) bytes += align256(l.size() * sizeof(Sum2Desc));
    for (auto& l : p.accum) bytes += align256(l.size() * sizeof(AccumDesc));
    host.assign(bytes, 0);
    dp.d_presum.clear();
    dp.d_combine.clear();
    dp.d_sums.clear();
    dp.d_accum.clear();
    size_t off = 0;
    auto put = [&](const void* src, size_t n) {
        if (n) std::memcpy(host.data() + off, src, n);
        void* d = base + off;
        off += align256(n);
        return d;
    };
    dp.d_leaves = static_cast<LeafDesc*>(put(p.leaves.data(), p.leaves.size() * sizeof(LeafDesc)));
    for (auto& l : p.presum) dp.d_presum.push_back(static_cast<PresumDesc*>(put(l.data(), l.size() * sizeof(PresumDesc))));
    for (auto& l : p.combine) dp.d_combine.push_back(static_cast<CombineDesc*>(put(l.data(), l.size() * sizeof(CombineDesc))));
    dp.d_nodes = static_cast<NodeDesc*>(put(p.nodes.data(), p.nodes.size() * sizeof(NodeDesc)));
    dp.d_pack = static_cast<PackDesc*>(put(p.pack.data(), p.pack.size() * sizeof(PackDesc)));
    dp.d_fb_leaves = static_cast<LeafDesc*>(put(p.fb_leaves.data(), p.fb_leaves.size() * sizeof(LeafDesc)));
    dp.d_pack8 = static_cast<Pack8Desc*>(put(p.pack8.data(), p.pack8.size() * sizeof(Pack8Desc)));
    dp.d_col1 = static_cast<ColDesc*>(put(p.col1.data(), p.col1.size() * sizeof(ColDesc)));
    dp.d_col2 = static_cast<ColDesc*>(put(p.col2.data(), p.col2.size() * sizeof(ColDesc)));
    dp.d_reduce = static_cast<ReduceDesc*>(put(p.reduce.data(), p.reduce.size() * sizeof(ReduceDesc)));
    for (auto& l : p.sums) dp.d_sums.push_back(static_cast<Sum2Desc*>(put(l.data(), l.size() * sizeof(Sum2Desc))));
    for (auto& l : p.accum)
        dp.d_accum.push_back(static_cast<AccumDesc*>(put(l.data(), l.size() * sizeof(AccumDesc))));
    return bytes;
}

ata_status_t upload_plan(DevicePlan& dp) {
    std::vector<unsigned char> host;
    const size_t bytes = layout_descriptors(dp, nullptr, host);
    if (bytes == 0) return ATA_OK;
    if (hipMalloc(&dp.d_buf, bytes) != hipSuccess) {
        dp.d_buf = nullptr;
        return ATA_ERR_OUT_OF_MEMORY;
    }
    layout_descriptors(dp, static_cast<unsigned char*>(dp.d_buf), host);
    return hip_status(hipMemcpy(dp.d_buf, host.data(), bytes, hipMemcpyHostToDevice));
}

bool valid_dtype(int d) { return d >= ATA_F64 && d <= ATA_F32_FP8E4M3; }

// Modes with a choice of leaf tile, and the tiles worth timing.
bool tiled_mode(int32_t mode) { return mode == MODE_BF16X3 || mode == MODE_FP8 || mode == MODE_F32; }
std::vector<int32_t> tile_candidates(int32_t mode) {
    if (mode == MODE_BF16X3) return {0, 1, 2, 3, 4};
    if (mode == MODE_F32) return {0, 2, 3};
    if (mode == MODE_FP8) return {0, 3};
    return {0};
}

// Leaf cutoff, depth cap and tile of one problem: explicit options win, then
// the autotune table, then the planner's defaults.
void choose(const ata_ctx* h, int32_t mode, int64_t m, int64_t n, int64_t& b, int32_t& depth,
            int32_t& tile, bool use_table = true) {
    b = h->popt.leaf_cutoff;
    depth = h->popt.max_depth;
    tile = tiled_mode(mode) ? h->popt.tile_cfg : 0;
    if (use_table && b <= 0 && depth < 0) {
        auto it = h->tune.find(TuneKey{mode, bucket(m), bucket(n)});
        if (it != h->tune.end()) {
            b = it->second.leaf_cutoff;
            depth = it->second.max_depth;
            if (tile < 0) tile = it->second.leaf_tile;
        }
    }
    if (tile < 0) tile = default_leaf_tile(mode, m, n);
    if (b <= 0) b = default_leaf_cutoff(mode, m, n, tile);
    if (depth < 0) depth = default_max_depth(mode, m);
}

// Bytes of auxiliary device memory one call needs (flags, norms, residual).
struct AuxLayout {
    size_t counter_off = 0, flags_off = 0, part_off = 0, nu_off = 0, res_work_off = 0, res_off = 0, total = 0;
};

AuxLayout aux_layout(const Plan& p, bool residual) {
    AuxLayout a;
    size_t off = 0;
    a.counter_off = off;                     // eight queue heads of a persistent leaf launch
    off += 256;
    a.flags_off = off;
    off += align256(std::max<size_t>(p.nodes.size(), 1));
    a.part_off = off;
    off += align256(sizeof(double) * (size_t)(p.fallback ? p.col_partial : 0));
    a.nu_off = off;
    off += align256(sizeof(double) * (size_t)(p.fallback ? p.n : 0));
    a.res_work_off = off;
    off += align256(sizeof(double) * (size_t)(residual ? residual_work_elems(p.m, p.n) : 0));
    a.res_off = off;
    off += align256(sizeof(double));
    a.total = off;
    return a;
}

// Does any column-norm pass 1 task also write a split-BF16 packing?
bool has_pack(const std::vector<ColDesc>& col1) {
    for (const auto& c : col1)
        if (c.pack) return true;
    return false;
}

// Leaf launch form: 1 = persistent, 0 = one workgroup per tile, -1 = the
// automatic choice (persistent for the 256 x 256 FP32 tile only).
bool persistent_for(int setting, const Plan& p) {
    if (setting >= 0) return setting == 1;
    return p.mode == MODE_F32 && p.tile_cfg >= 2;
}

// Does the plan's workspace fit in the device memory that is free (the arena
// the handle already holds counts as free), with 1 GiB to spare?  The GPU
// keeps every Strassen level's sums and products at once (a level's products
// run concurrently), so the workspace grows about 7/4 per level: a plan for a
// large matrix gets fewer levels rather than an allocation failure.
bool fits_device(const ata_ctx* h, int64_t arena_elems, int64_t elem_bytes) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return true;
    const double need = (double)arena_elems * (double)elem_bytes;
    return need + (double)(1ull << 30) <= (double)free_b + (double)h->arena_cap;
}
bool fits_device(const ata_ctx* h, const Plan& p) { return fits_device(h, p.arena_elems, p.elem_bytes()); }

int64_t max_arena(const std::vector<Plan>& st) {
    int64_t a = 0;
    for (const auto& q : st) a = std::max(a, q.arena_elems);
    return a;
}

// The bounded-workspace (staged) plan of a key, with the Strassen depth
// lowered until the largest stage fits the device; stage 0 goes into dp,
// the others into dp.stages, each with its descriptors uploaded.
ata_status_t build_staged(const ata_ctx* h, const PlanKey& k, DevicePlan& dp) {
    PlanOptions o;
    o.leaf_cutoff = k.b;
    o.max_depth = k.depth;
    o.spread_tau = k.fb ? h->popt.spread_tau : 0.0;
    o.tile_cfg = k.tile_cfg;
    o.split_target = k.split;
    o.slots = k.slots;
    o.bounded = true;
    std::vector<Plan> st;
    try {
        st = make_staged_plan(k.mode, k.m, k.n, k.lda, o);
        while (st[0].stats.max_levels > 0 && !fits_device(h, max_arena(st), st[0].elem_bytes())) {
            o.max_depth = st[0].stats.max_levels - 1;
            st = make_staged_plan(k.mode, k.m, k.n, k.lda, o);
        }
        if (st[0].fallback) {
            fuse_pack_into_norms(st[0], st[0].col1);
            fuse_norms_into_quant(st[0], st[0].col1, st[0].col2, st[0].col_partial);
        }
    } catch (const std::invalid_argument&) {
        return ATA_ERR_INVALID_VALUE;
    } catch (const std::length_error&) {
        return ATA_ERR_NOT_SUPPORTED;
    } catch (const std::exception&) {
        return ATA_ERR_INTERNAL;
    }
    dp.stage_arena_elems = max_arena(st);
    dp.plan = std::move(st[0]);
    ata_status_t s = upload_plan(dp);
    for (size_t i = 1; s == ATA_OK && i < st.size(); ++i) {
        auto sp = std::make_unique<DevicePlan>();
        sp->plan = std::move(st[i]);
        s = upload_plan(*sp);
        dp.stages.push_back(std::move(sp));
    }
    return s;
}


// The plan of one Gram product for a plan-cache key, with the Strassen depth
// lowered one level at a time until `fits` accepts the plan (a plan without
// Strassen levels is returned whether it fits or not).
template <class Fits>
ata_status_t build_gram_plan(const ata_ctx* h, const PlanKey& k, Fits fits, Plan& out) {
    PlanOptions o;
    o.leaf_cutoff = k.b;
    o.max_depth = k.depth;
    o.spread_tau = k.fb ? h->popt.spread_tau : 0.0;
    o.tile_cfg = k.tile_cfg;
    o.split_target = k.split;
    o.fuse_presum = k.fuse;
    o.variant = k.variant;
    o.slots = k.slots;
    o.overlap = k.overlap;
    o.fuse_combine = k.fuse_combine;
    try {
        out = make_plan(k.mode, k.m, k.n, k.lda, o);
        while (out.stats.max_levels > 0 && !fits(out)) {
            o.max_depth = out.stats.max_levels - 1;
            out = make_plan(k.mode, k.m, k.n, k.lda, o);
        }
        if (out.fallback) {
            fuse_pack_into_norms(out, out.col1);
            fuse_norms_into_quant(out, out.col1, out.col2, out.col_partial);
        }
    } catch (const std::invalid_argument&) {
        return ATA_ERR_INVALID_VALUE;
    } catch (const std::length_error&) {
        return ATA_ERR_NOT_SUPPORTED;
    } catch (const std::exception&) {
        return ATA_ERR_INTERNAL;
    }
    return ATA_OK;
}

// Resident leaf workgroups of the device (256 CUs) for the tail balancer,
// or 0 when it is off.
int64_t tail_slots(const ata_ctx* h, int32_t mode, int32_t tile_cfg) {
    return h->balance_tail ? (int64_t)leaf_blocks_per_cu(mode, tile_cfg) * 256 : 0;
}

// Whether a plan combines its last Strassen level in the leaf epilogues:
// asked for, Strassen's form, and a leaf tile built for it (the 256 x 256
// four-wave FP32 and split-BF16 tiles are not).
bool combine_in_epilogue(const ata_ctx* h, int32_t mode, int32_t tile_cfg) {
    return h->popt.fuse_combine && h->popt.variant == 0 &&
           !((mode == MODE_F32 || mode == MODE_BF16X3) && tile_cfg == 3);
}

void fill_report(ata_report_t& r, const Plan& p) {
    r.m = p.m;
    r.n = p.n;
    r.lda = p.lda;
    r.dtype = p.mode;
    r.strassen_levels = p.stats.max_levels;
    r.leaf_cutoff = p.b;
    r.ata_nodes = p.stats.ata_nodes;
    r.syrk_leaves = p.stats.syrk_leaves;
    r.gemm_leaves = p.stats.gemm_leaves;
    r.strassen_nodes = p.stats.strassen_nodes;
    r.multiplications = p.stats.mults;
    r.workspace_bytes = p.arena_elems * p.elem_bytes();
    r.kernel_launches = p.launches();
    r.flagged_nodes = -1;
    r.residual = -1.0;
    r.leaf_tile = p.tile_cfg;
    r.leaf_persistent = 0;
    r.tail_split_leaves = p.tail_leaves;
    r.tail_split_chunks = p.tail_chunks;
    r.leaf_rounds = p.leaves.empty() ? 0 : 1;
    if (!p.round_tiles.empty()) {
        r.leaf_rounds = 0;
        for (size_t i = 0; i + 1 < p.round_tiles.size(); ++i)
            r.leaf_rounds += p.round_tiles[i + 1] > p.round_tiles[i] ? 1 : 0;
    }
}

}  // namespace

extern "C" {

const char* ata_status_string(ata_status_t s) {
    switch (s) {
        case ATA_OK: return "ATA_OK";
        case ATA_ERR_INVALID_VALUE: return "ATA_ERR_INVALID_VALUE";
        case ATA_ERR_NOT_SUPPORTED: return "ATA_ERR_NOT_SUPPORTED";
        case ATA_ERR_OUT_OF_MEMORY: return "ATA_ERR_OUT_OF_MEMORY";
        case ATA_ERR_HIP: return "ATA_ERR_HIP";
        case ATA_ERR_INTERNAL: return "ATA_ERR_INTERNAL";
    }
    return "ATA_ERR_UNKNOWN";
}

ata_status_t ata_create(ata_handle_t* out) {
    if (!out) return ATA_ERR_INVALID_VALUE;
    *out = nullptr;
    int dev = 0, count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return ATA_ERR_HIP;
    if (hipGetDevice(&dev) != hipSuccess) return ATA_ERR_HIP;
    ata_ctx* h = new (std::nothrow) ata_ctx;
    if (!h) return ATA_ERR_OUT_OF_MEMORY;
    h->device = dev;
    h->popt.tile_cfg = -1;                 // automatic: autotune table, else by shape
    if (dev < kMaxDevices && scratch_address(dev, h->scratch) != ATA_OK) {
        delete h;
        return ATA_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) h->arch = prop.gcnArchName;
    *out = h;
    return ATA_OK;
}

ata_status_t ata_destroy(ata_handle_t h) {
    if (!h) return ATA_OK;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    h->batches.clear();
    h->plans.clear();
    if (h->batch_stream) (void)hipStreamDestroy(h->batch_stream);
    if (h->batch_in) (void)hipEventDestroy(h->batch_in);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    if (h->join_ev) (void)hipEventDestroy(h->join_ev);
    clear_events(h);
    if (h->arena) (void)hipFree(h->arena);
    if (h->aux) (void)hipFree(h->aux);
    if (h->tmp) (void)hipFree(h->tmp);
    if (h->eq) (void)hipFree(h->eq);
    for (void* p : h->retired) (void)hipFree(p);
    delete h;
    return ATA_OK;
}

ata_status_t ata_set_option(ata_handle_t h, ata_option_t key, double value) {
    if (!h) return ATA_ERR_INVALID_VALUE;
    switch (key) {
        case ATA_OPT_LEAF_CUTOFF:
            if (value < 0) return ATA_ERR_INVALID_VALUE;
            h->popt.leaf_cutoff = (int64_t)value;
            return ATA_OK;
        case ATA_OPT_MAX_STRASSEN_DEPTH:
            if (value < -1 || value > 64) return ATA_ERR_INVALID_VALUE;
            h->popt.max_depth = (int32_t)value;
            return ATA_OK;
        case ATA_OPT_SPREAD_TAU:
            h->popt.spread_tau = value;
            return ATA_OK;
        case ATA_OPT_RESIDUAL:
            h->residual = value != 0.0;
            return ATA_OK;
        case ATA_OPT_WORKSPACE_LIMIT:
            if (value < 0) return ATA_ERR_INVALID_VALUE;
            h->ws_limit = (int64_t)value;
            return ATA_OK;
        case ATA_OPT_RESIDUAL_SEED:
            h->seed = (uint64_t)value;
            return ATA_OK;
        case ATA_OPT_LEAF_TILE:
            if (value != -1 && value != 0 && value != 1 && value != 2 && value != 3 && value != 4)
                return ATA_ERR_INVALID_VALUE;
            h->popt.tile_cfg = (int32_t)value;
            return ATA_OK;
        case ATA_OPT_BATCH_GRAPH:
            h->batch_graph = value != 0.0;
            return ATA_OK;
        case ATA_OPT_BATCH_PERSISTENT:
            if (value != -1.0 && value != 0.0 && value != 1.0) return ATA_ERR_INVALID_VALUE;
            h->batch_persistent = (int)value;
            return ATA_OK;
        case ATA_OPT_XCD_CHUNK:
            if (value < 1 || value > 4096) return ATA_ERR_INVALID_VALUE;
            h->chunk = (int)value;
            return ATA_OK;
        case ATA_OPT_TILE_BAND:
            if (value < 1 || value > 4096) return ATA_ERR_INVALID_VALUE;
            h->band = (int)value;
            return ATA_OK;
        case ATA_OPT_EQUILIBRATE:
            h->equilibrate = value != 0.0;
            return ATA_OK;
        case ATA_OPT_LEAF_PERSISTENT:
            if (value != -1.0 && value != 0.0 && value != 1.0) return ATA_ERR_INVALID_VALUE;
            h->leaf_persistent = (int)value;
            return ATA_OK;
        case ATA_OPT_FUSE_PRESUM:
            h->popt.fuse_presum = value != 0.0;
            return ATA_OK;
        case ATA_OPT_BALANCE_TAIL:
            h->balance_tail = value != 0.0;
            return ATA_OK;
        case ATA_OPT_STRASSEN_FORM:
            if (value != 0.0 && value != 1.0) return ATA_ERR_INVALID_VALUE;
            h->popt.variant = (int32_t)value;
            return ATA_OK;
        case ATA_OPT_BATCH_USE_TABLE:
            h->batch_use_table = value != 0.0;
            return ATA_OK;
        case ATA_OPT_SPLIT_TARGET:
            if (value < 0 || value > 1e9) return ATA_ERR_INVALID_VALUE;
            h->split_target = (int64_t)value;
            return ATA_OK;
        case ATA_OPT_OVERLAP:
            if (value != -1.0 && value != 0.0 && value != 1.0) return ATA_ERR_INVALID_VALUE;
            h->overlap = (int)value;
            return ATA_OK;
        case ATA_OPT_BOUNDED_WORKSPACE:
            h->bounded = value != 0.0;
            return ATA_OK;
        case ATA_OPT_FUSE_COMBINE:
            h->popt.fuse_combine = value != 0.0;
            return ATA_OK;
        case ATA_OPT_PROFILE:
            if (h->events_used) (void)drain_events(h);
            h->profile = value != 0.0;
            h->profiled_calls = 0;
            for (double& x : h->phase_ms) x = 0.0;
            return ATA_OK;
    }
    return ATA_ERR_INVALID_VALUE;
}

ata_status_t ata_plan_query(int64_t m, int64_t n, ata_dtype_t dtype, int64_t leaf_cutoff,
                            int32_t max_depth, ata_report_t* info, ata_leaf_t* leaves,
                            int64_t cap, int64_t* n_leaves) {
    if (!valid_dtype(dtype) || m < 0 || n < 0 || cap < 0 || (cap > 0 && !leaves))
        return ATA_ERR_INVALID_VALUE;
    PlanOptions o;
    o.leaf_cutoff = leaf_cutoff > 0 ? leaf_cutoff : 0;
    o.max_depth = max_depth;
    o.spread_tau = 0.0;
    Plan p;
    try {
        p = make_plan((int32_t)dtype, m, n, std::max<int64_t>(1, n), o);
    } catch (const std::length_error&) {
        return ATA_ERR_NOT_SUPPORTED;
    } catch (const std::exception&) {
        return ATA_ERR_INVALID_VALUE;
    }
    if (info) fill_report(*info, p);
    if (n_leaves) *n_leaves = (int64_t)p.leaves.size();
    for (int64_t i = 0; i < cap && i < (int64_t)p.leaves.size(); ++i) {
        const LeafDesc& L = p.leaves[i];
        ata_leaf_t& o2 = leaves[i];
        o2.kind = L.kind;
        o2.depth = L.depth;
        o2.rows = L.rows;
        o2.cols = L.cols;
        o2.contraction = L.K;
        o2.out_row0 = L.out_kind == OUT_PACKED ? L.out_row0 : -1;
        o2.out_col0 = L.out_kind == OUT_PACKED ? L.out_col0 : -1;
        o2.ksplit = L.ksplit > 1 ? L.ksplit : 1;
        o2.pad_ = 0;
    }
    return ATA_OK;
}

namespace {

// Six profiling events for one call (null when profiling is off).
ata_status_t take_events(ata_ctx* h, hipEvent_t*& ev) {
    ev = nullptr;
    if (!h->profile) return ATA_OK;
    if (h->events_used + EVENTS_PER_CALL > 4096 && drain_events(h) != hipSuccess) return ATA_ERR_HIP;
    while (h->events.size() < h->events_used + EVENTS_PER_CALL) {
        hipEvent_t x;
        if (hipEventCreate(&x) != hipSuccess) return ATA_ERR_HIP;
        h->events.push_back(x);
    }
    ev = h->events.data() + h->events_used;
    h->events_used += EVENTS_PER_CALL;
    return ATA_OK;
}

}  // namespace

namespace {

// The leaf products of a plan: one launch, or one per launch round when the
// plan combines its last Strassen level in the leaf epilogues (the rounds
// run in order on `st`).
hipError_t launch_plan_leaves(const ata_ctx* h, const DevicePlan& dp, const void* A, void* C, void* arena,
                              const uint8_t* flags, hipStream_t st, const BatchPtrs* lp, const void* B = nullptr) {
    const Plan& p = dp.plan;
    if (p.round_tiles.empty())
        return launch_leaves(p.mode, p.tile_cfg, dp.d_leaves, (int)p.leaves.size(), p.total_tiles, A, C, arena,
                             flags, h->chunk, h->band, st, lp, B);
    hipError_t e = hipSuccess;
    for (size_t r = 0; e == hipSuccess && r + 1 < p.round_tiles.size(); ++r)
        e = launch_leaves_epi(p.mode, p.tile_cfg, dp.d_leaves, (int)p.leaves.size(),
                              p.round_tiles[r + 1] - p.round_tiles[r], A, C, arena, flags, h->chunk, h->band, st,
                              lp, B, p.round_tiles[r]);
    return e;
}

// Enqueue every phase of a single-problem plan on `st`: column norms and
// spread flags, pre-sums level by level, packing or quantisation, the leaf
// launch, the FP64 fallback, the split-K reduce, the combines bottom-up, and
// the optional residual probe.  `arena` and `aux` (laid out by aux_layout)
// are the call's workspace; `ev` holds six profiling events or is null.
hipError_t enqueue_gram(const ata_ctx* h, const DevicePlan& dp, const void* A, void* C_packed, void* arena,
                        unsigned char* aux, const AuxLayout& ax, bool residual, hipStream_t st, hipEvent_t* ev,
                        bool& persistent, bool mark_end = true, bool overlap = false) {
    const Plan& p = dp.plan;
    const int32_t mode = p.mode;
    // two blocks of eight queue heads: the A-only leaves' launch on the side
    // stream, and the caller stream's launch
    BatchPtrs pq{nullptr, nullptr, reinterpret_cast<unsigned long long*>(aux + ax.counter_off), 0};
    BatchPtrs pq2 = pq;
    pq2.counter += 8;
    const BatchPtrs* lp = nullptr;
    const BatchPtrs* lp2 = nullptr;
    if (persistent_for(h->leaf_persistent, p)) {
        pq.persistent_blocks = pq2.persistent_blocks = (int64_t)leaf_blocks_per_cu(mode, p.tile_cfg) * 256;
        lp = &pq;
        lp2 = &pq2;
    }
    persistent = lp != nullptr;
    const bool ov = overlap && p.indep_tiles > 0 && h->side && h->fork_ev && h->join_ev;
    uint8_t* flags = aux + ax.flags_off;
    double* partial = reinterpret_cast<double*>(aux + ax.part_off);
    double* nu = reinterpret_cast<double*>(aux + ax.nu_off);
    double* res_work = reinterpret_cast<double*>(aux + ax.res_work_off);
    double* res = reinterpret_cast<double*>(aux + ax.res_off);
    hipError_t e = hipSuccess;
    auto mark = [&](int i) {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[i], st);
    };
    mark(0);
    const int32_t ps = p.pack_split, q0 = p.pack8_norm, qs = std::max(p.pack8_split, q0);
    if (p.fallback) {
        // FP8: the quantisations of A's column slices write the norm partials
        if (q0 > 0)
            e = launch_quant8(dp.d_pack8, q0, p.pack8[q0 - 1].elem_begin + p.pack8[q0 - 1].elems, A, arena, flags,
                              st, nullptr, nullptr, partial);
        if (e == hipSuccess)
            e = launch_colnorms(dp.d_col1, (int)p.col1.size(), p.col1.back().elem_begin + p.col1.back().elems,
                                dp.d_col2, (int)p.col2.size(), p.col2.back().elem_begin + p.col2.back().elems,
                                static_cast<const float*>(A), nullptr, partial, nu, st, arena, has_pack(p.col1));
        if (e == hipSuccess)
            e = launch_flags(nu, dp.d_nodes, (int)p.nodes.size(), h->popt.spread_tau * h->popt.spread_tau, flags, st);
    }
    mark(1);
    // packings and quantisations of views of A (the A-only leaves read them)
    if (e == hipSuccess && ps > 0)
        e = launch_pack(dp.d_pack, ps, p.pack[ps - 1].elem_begin + p.pack[ps - 1].elems, A, arena, flags, st);
    if (e == hipSuccess && qs > q0)
        e = launch_quant8(dp.d_pack8 + q0, qs - q0, p.pack8[qs - 1].elem_begin + p.pack8[qs - 1].elems, A, arena,
                          flags, st);
    if (ov && e == hipSuccess) {
        // the leaves that read only A, and the FP64 fallback, beside the pre-sums
        e = hipEventRecord(h->fork_ev, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->side, h->fork_ev, 0);
        if (e == hipSuccess)
            e = launch_leaves(mode, p.tile_cfg, dp.d_leaves, (int)p.leaves.size(), p.indep_tiles, A, C_packed, arena,
                              flags, h->chunk, h->band, h->side, lp);
        if (e == hipSuccess && !p.fb_leaves.empty())
            e = launch_fallback_leaves(dp.d_fb_leaves, (int)p.fb_leaves.size(), p.fb_tiles, A, C_packed, arena,
                                       flags, h->chunk, h->band, h->side);
        if (e == hipSuccess) e = hipEventRecord(h->join_ev, h->side);
    }
    for (size_t l = 0; e == hipSuccess && l < p.sums.size(); ++l) {
        const auto& lv = p.sums[l];
        if (!lv.empty())
            e = launch_sum2(mode, dp.d_sums[l], (int)lv.size(), lv.back().elem_begin + lv.back().elems, A, arena,
                            flags, st);
    }
    // (a bounded-workspace stage's resident subtree starts below the top,
    // so its upper pre-sum levels are empty)
    for (size_t l = 0; e == hipSuccess && l < p.presum.size(); ++l) {
        const auto& lv = p.presum[l];
        if (!lv.empty())
            e = launch_presum(mode, dp.d_presum[l], (int)lv.size(), lv.back().elem_begin + lv.back().elems,
                              A, arena, flags, st);
    }
    if (e == hipSuccess && (int32_t)p.pack.size() > ps)
        e = launch_pack(dp.d_pack + ps, (int)p.pack.size() - ps, p.pack.back().elem_begin + p.pack.back().elems,
                        A, arena, flags, st);
    if (e == hipSuccess && (int32_t)p.pack8.size() > qs)
        e = launch_quant8(dp.d_pack8 + qs, (int)p.pack8.size() - qs,
                          p.pack8.back().elem_begin + p.pack8.back().elems, A, arena, flags, st);
    mark(2);
    if (ov) {
        if (e == hipSuccess)
            e = launch_leaves(mode, p.tile_cfg, dp.d_leaves, (int)p.leaves.size(), p.total_tiles - p.indep_tiles, A,
                              C_packed, arena, flags, h->chunk, h->band, st, lp2, nullptr, p.indep_tiles);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, h->join_ev, 0);
    } else {
        if (e == hipSuccess) e = launch_plan_leaves(h, dp, A, C_packed, arena, flags, st, lp);
        if (e == hipSuccess && !p.fb_leaves.empty())
            e = launch_fallback_leaves(dp.d_fb_leaves, (int)p.fb_leaves.size(), p.fb_tiles, A, C_packed,
                                       arena, flags, h->chunk, h->band, st);
    }
    if (e == hipSuccess && !p.reduce.empty())
        e = launch_reduce(mode, dp.d_reduce, (int)p.reduce.size(), p.reduce.back().elem_begin + p.reduce.back().elems,
                          C_packed, arena, flags, st);
    mark(3);
    for (size_t l = 0; e == hipSuccess && l < p.combine.size(); ++l) {
        const auto& lv = p.combine[l];
        if (!lv.empty())
            e = launch_combine(mode, dp.d_combine[l], (int)lv.size(), lv.back().elem_begin + lv.back().elems,
                               C_packed, arena, flags, st);
    }
    for (size_t l = 0; e == hipSuccess && l < p.accum.size(); ++l) {
        const auto& lv = p.accum[l];
        if (!lv.empty())
            e = launch_accum(mode, dp.d_accum[l], (int)lv.size(), lv.back().elem_begin + lv.back().elems, C_packed,
                             arena, flags, st);
    }
    mark(4);
    if (e == hipSuccess && residual)
        e = launch_residual(mode, A, p.m, p.n, p.lda, C_packed, h->seed, res_work, res, st);
    if (mark_end) mark(5);
    return e;
}

// A staged (bounded-workspace) plan: stage 0 with the column norms and
// flags, then every later stage on the same arena and flags; the residual
// probe after the last stage.  Profiling: phases 0-3 are stage 0's, phase 4
// runs from stage 0's combines to the end.
hipError_t enqueue_staged(const ata_ctx* h, const DevicePlan& dp, const void* A, void* C_packed, void* arena,
                          unsigned char* aux, const AuxLayout& ax, bool residual, hipStream_t st, hipEvent_t* ev,
                          bool& persistent) {
    hipError_t e = enqueue_gram(h, dp, A, C_packed, arena, aux, ax, false, st, ev, persistent, false);
    for (const auto& sp : dp.stages) {
        bool pers = false;
        if (e == hipSuccess) e = enqueue_gram(h, *sp, A, C_packed, arena, aux, ax, false, st, nullptr, pers);
    }
    const Plan& p = dp.plan;
    if (e == hipSuccess && residual)
        e = launch_residual(p.mode, A, p.m, p.n, p.lda, C_packed, h->seed,
                            reinterpret_cast<double*>(aux + ax.res_work_off),
                            reinterpret_cast<double*>(aux + ax.res_off), st);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[5], st);
    return e;
}

}  // namespace

namespace {

// Column equilibration (an alternative to the FP64 fallback for ill-scaled
// columns): scale column j by 2^-e_j so that every column norm lies in
// [0.5, 1), run the plan on the scaled copy (no spread check needed: the
// norms now differ by less than 2x), and scale C_ij back by 2^(e_i + e_j).
// All scalings are exact powers of two, so in exact arithmetic the result is
// A^T A itself; each entry's rounding error becomes relative to
// ||a_i|| ||a_j|| instead of to the largest columns.
ata_status_t gram_equilibrated(ata_ctx* h, const void* A, int64_t m, int64_t n, int64_t lda, ata_dtype_t dtype,
                               void* C_packed, void* stream) {
    const auto key = std::make_tuple(m, n, lda);
    auto it = h->eq_plans.find(key);
    if (it == h->eq_plans.end()) {
        auto dp = std::make_unique<DevicePlan>();
        dp->plan.m = m;
        dp->plan.n = n;
        dp->plan.lda = lda;
        build_colnorm_tasks(&m, &n, &lda, 1, dp->plan.col1, dp->plan.col2, &dp->plan.col_partial);
        const ata_status_t s = upload_plan(*dp);
        if (s != ATA_OK) return s;
        it = h->eq_plans.emplace(key, std::move(dp)).first;
    }
    const DevicePlan& ep = *it->second;
    const Plan& q = ep.plan;
    const size_t ap_b = align256(sizeof(float) * (size_t)(m * n));
    const size_t part_b = align256(sizeof(double) * (size_t)std::max<int64_t>(q.col_partial, 1));
    const size_t nu_b = align256(sizeof(double) * (size_t)n);
    const size_t e_b = align256(sizeof(int) * (size_t)n);
    ata_status_t s = ensure(h, h->eq, h->eq_cap, ap_b + part_b + nu_b + e_b);
    if (s != ATA_OK) return s;
    unsigned char* base = static_cast<unsigned char*>(h->eq);
    float* Ap = reinterpret_cast<float*>(base);
    double* partial = reinterpret_cast<double*>(base + ap_b);
    double* nu = reinterpret_cast<double*>(base + ap_b + part_b);
    int* e = reinterpret_cast<int*>(base + ap_b + part_b + nu_b);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t err = launch_colnorms(ep.d_col1, (int)q.col1.size(), q.col1.back().elem_begin + q.col1.back().elems,
                                     ep.d_col2, (int)q.col2.size(), q.col2.back().elem_begin + q.col2.back().elems,
                                     static_cast<const float*>(A), nullptr, partial, nu, st);
    if (err == hipSuccess) err = launch_eq_scale(static_cast<const float*>(A), m, n, lda, nu, Ap, e, st);
    if (err != hipSuccess) return ATA_ERR_HIP;
    // the plan on the scaled copy, without the spread check
    const double tau = h->popt.spread_tau;
    h->equilibrate = false;
    h->popt.spread_tau = 0.0;
    s = ata_gram(h, Ap, m, n, n, dtype, C_packed, stream);
    h->equilibrate = true;
    h->popt.spread_tau = tau;
    if (s != ATA_OK) return s;
    return launch_eq_unscale(static_cast<float*>(C_packed), n, e, st) == hipSuccess ? ATA_OK : ATA_ERR_HIP;
}

}  // namespace

ata_status_t ata_gram(ata_handle_t h, const void* A, int64_t m, int64_t n, int64_t lda,
                      ata_dtype_t dtype, void* C_packed, void* stream) {
    if (!h || !valid_dtype(dtype) || m < 0 || n < 0 || lda < std::max<int64_t>(1, n))
        return ATA_ERR_INVALID_VALUE;
    if (n > 0 && !C_packed) return ATA_ERR_INVALID_VALUE;
    if (n > 0 && m > 0 && !A) return ATA_ERR_INVALID_VALUE;
    const size_t es = dtype == ATA_F64 ? 8 : 4;
    if (n > 0 && m > 0) {
        const uintptr_t a0 = (uintptr_t)A, a1 = a0 + (size_t)((m - 1) * lda + n) * es;
        const uintptr_t c0 = (uintptr_t)C_packed, c1 = c0 + (size_t)(n * (n + 1) / 2) * es;
        if (a0 < c1 && c0 < a1) return ATA_ERR_INVALID_VALUE;
    }
    if (n == 0) {
        h->report = ata_report_t{};
        h->report.m = m;
        h->report.lda = lda;
        h->report.dtype = dtype;
        h->report.flagged_nodes = -1;
        h->report.residual = -1.0;
        h->pending_flags = h->pending_residual = false;
        return ATA_OK;
    }
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    note_capture(h, stream);
    h->spread_plan = nullptr;
    const int32_t mode = (int32_t)dtype;
    if (h->equilibrate && mode != MODE_F64 && m > 0) return gram_equilibrated(h, A, m, n, lda, dtype, C_packed, stream);
    int64_t b;
    int32_t depth, tile_cfg;
    choose(h, mode, m, n, b, depth, tile_cfg);
    const bool fb = mode != MODE_F64 && h->popt.spread_tau > 0 && m > 0;
    const int64_t slots = tail_slots(h, mode, tile_cfg);
    const bool bounded = h->bounded;
    const bool overlap = !bounded && h->overlap == 1;
    const PlanKey key{mode, m, n, lda, b, depth, fb, tile_cfg, h->split_target,
                      bounded ? false : h->popt.fuse_presum, bounded ? 0 : h->popt.variant, slots, bounded,
                      overlap, !bounded && combine_in_epilogue(h, mode, tile_cfg)};
    auto it = h->plans.find(key);
    if (it == h->plans.end()) {
        auto dp = std::make_unique<DevicePlan>();
        if (bounded) {
            const ata_status_t s = build_staged(h, key, *dp);
            if (s != ATA_OK) return s;
        } else {
            const ata_status_t s =
                build_gram_plan(h, key, [h](const Plan& q) { return fits_device(h, q); }, dp->plan);
            if (s != ATA_OK) return s;
            const ata_status_t su = upload_plan(*dp);
            if (su != ATA_OK) return su;
        }
        it = h->plans.emplace(key, std::move(dp)).first;
    }
    DevicePlan& dp = *it->second;
    const Plan& p = dp.plan;
    const AuxLayout ax = aux_layout(p, h->residual);
    const size_t arena_bytes = (size_t)dp.arena_elems() * (size_t)p.elem_bytes();
    if (h->ws_limit > 0 && (int64_t)(arena_bytes + ax.total) > h->ws_limit) return ATA_ERR_OUT_OF_MEMORY;
    const size_t old_cap = h->arena_cap;
    ata_status_t s = ensure(h, h->arena, h->arena_cap, std::max<size_t>(arena_bytes, 256));
    if (s != ATA_OK) return s;
    if (h->arena_cap != old_cap) ++h->arena_gen;
    s = ensure(h, h->aux, h->aux_cap, ax.total);
    if (s != ATA_OK) return s;

    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char* aux = static_cast<unsigned char*>(h->aux);
    hipEvent_t* ev = nullptr;
    if (take_events(h, ev) != ATA_OK) return ATA_ERR_HIP;
    if (overlap && p.indep_tiles > 0 && !h->side) {
        if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) {
            h->side = nullptr;
            return ATA_ERR_HIP;
        }
        if (hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming) != hipSuccess)
            return ATA_ERR_HIP;
    }
    bool persistent = false;
    const hipError_t eq = dp.stages.empty()
                              ? enqueue_gram(h, dp, A, C_packed, h->arena, aux, ax, h->residual, st, ev, persistent,
                                             true, overlap)
                              : enqueue_staged(h, dp, A, C_packed, h->arena, aux, ax, h->residual, st, ev, persistent);
    if (eq != hipSuccess) return ATA_ERR_HIP;

    fill_report(h->report, p);
    h->report.leaf_persistent = persistent ? 1 : 0;
    h->report.overlapped = overlap && p.indep_tiles > 0 && dp.stages.empty() ? 1 : 0;
    if (h->report.overlapped) h->report.kernel_launches += 1;
    if (!dp.stages.empty()) {
        h->report.workspace_bytes = (int64_t)arena_bytes;
        for (const auto& sp : dp.stages) h->report.kernel_launches += sp->plan.launches();
    }
    h->last_stream = st;
    h->pending_flags = p.fallback;
    h->pending_residual = h->residual;
    h->last_flags = aux + ax.flags_off;
    h->last_residual = reinterpret_cast<double*>(aux + ax.res_off);
    h->last_nodes = (int64_t)p.nodes.size();
    if (p.fallback) {
        h->spread_plan = &dp;
        h->spread_nu = reinterpret_cast<double*>(aux + ax.nu_off);
        h->spread_flags = aux + ax.flags_off;
        h->spread_stream = st;
    }
    return ATA_OK;
}

namespace {

// Lay a plan out in the static workspace: descriptors, then the arena, then
// the auxiliary block.  Returns the bytes it needs.
size_t layout_static(StaticPlan& sp, unsigned char* base) {
    const Plan& p = sp.dp.plan;
    const size_t desc = align256(layout_descriptors(sp.dp, base, sp.blob));
    sp.arena_off = desc;
    sp.aux_off = sp.arena_off + align256((size_t)p.arena_elems * (size_t)p.elem_bytes());
    sp.total = sp.aux_off + aux_layout(p, false).total;
    return sp.total;
}

}  // namespace

ata_status_t ata_gram_noalloc(ata_handle_t h, const void* A, int64_t m, int64_t n, int64_t lda,
                              ata_dtype_t dtype, void* C_packed, void* stream) {
    if (!h || !valid_dtype(dtype) || m < 0 || n < 0 || lda < std::max<int64_t>(1, n))
        return ATA_ERR_INVALID_VALUE;
    if (n > 0 && !C_packed) return ATA_ERR_INVALID_VALUE;
    if (n > 0 && m > 0 && !A) return ATA_ERR_INVALID_VALUE;
    const size_t es = dtype == ATA_F64 ? 8 : 4;
    if (n > 0 && m > 0) {
        const uintptr_t a0 = (uintptr_t)A, a1 = a0 + (size_t)((m - 1) * lda + n) * es;
        const uintptr_t c0 = (uintptr_t)C_packed, c1 = c0 + (size_t)(n * (n + 1) / 2) * es;
        if (a0 < c1 && c0 < a1) return ATA_ERR_INVALID_VALUE;
    }
    const int32_t mode = (int32_t)dtype;
    if (h->residual || (h->equilibrate && mode != MODE_F64)) return ATA_ERR_NOT_SUPPORTED;
    h->report = ata_report_t{};
    h->report.m = m;
    h->report.lda = lda;
    h->report.dtype = dtype;
    h->report.flagged_nodes = -1;
    h->report.residual = -1.0;
    h->pending_flags = h->pending_residual = false;
    h->spread_plan = nullptr;
    if (n == 0) return ATA_OK;
    if (!h->scratch) return ATA_ERR_NOT_SUPPORTED;
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    int64_t b;
    int32_t depth, tile_cfg;
    choose(h, mode, m, n, b, depth, tile_cfg);
    const bool fb = mode != MODE_F64 && h->popt.spread_tau > 0 && m > 0;
    const PlanKey key{mode, m, n, lda, b, depth, fb, tile_cfg, h->split_target, h->popt.fuse_presum,
                      h->popt.variant, tail_slots(h, mode, tile_cfg), false, false,
                      combine_in_epilogue(h, mode, tile_cfg)};
    const size_t limit = h->ws_limit > 0 ? std::min<size_t>((size_t)h->ws_limit, ATA_NOALLOC_SCRATCH_BYTES)
                                         : (size_t)ATA_NOALLOC_SCRATCH_BYTES;
    auto it = h->static_plans.find(key);
    if (it == h->static_plans.end()) {
        auto sp = std::make_unique<StaticPlan>();
        auto fits = [&](const Plan& q) {
            StaticPlan t;
            t.dp.plan = q;
            return layout_static(t, h->scratch) <= limit;
        };
        ata_status_t s = build_gram_plan(h, key, fits, sp->dp.plan);
        if (s != ATA_OK) return s;
        if (!fits(sp->dp.plan) && (key.split != 0 || key.slots != 0)) {
            // without split-K partials and tail cuts
            PlanKey k2 = key;
            k2.split = 0;
            k2.slots = 0;
            s = build_gram_plan(h, k2, fits, sp->dp.plan);
            if (s != ATA_OK) return s;
        }
        if (layout_static(*sp, h->scratch) > limit) return ATA_ERR_OUT_OF_MEMORY;
        it = h->static_plans.emplace(key, std::move(sp)).first;
    }
    StaticPlan& sp = *it->second;
    const Plan& p = sp.dp.plan;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char* aux = h->scratch + sp.aux_off;
    hipError_t e = hipSuccess;
    if (!sp.blob.empty())
        e = hipMemcpyAsync(h->scratch, sp.blob.data(), sp.blob.size(), hipMemcpyHostToDevice, st);
    bool persistent = false;
    if (e == hipSuccess)
        e = enqueue_gram(h, sp.dp, A, C_packed, h->scratch + sp.arena_off, aux, aux_layout(p, false), false, st,
                         nullptr, persistent);
    if (e != hipSuccess) return ATA_ERR_HIP;
    fill_report(h->report, p);
    h->report.leaf_persistent = persistent ? 1 : 0;
    return ATA_OK;
}

ata_status_t ata_residual(ata_handle_t h, const void* A, int64_t m, int64_t n, int64_t lda,
                          ata_dtype_t dtype, const void* C_packed, uint64_t seed, double* result,
                          void* stream) {
    if (!h || !result || !valid_dtype(dtype) || m < 0 || n < 0 || lda < std::max<int64_t>(1, n))
        return ATA_ERR_INVALID_VALUE;
    if (n > 0 && (!C_packed || (m > 0 && !A))) return ATA_ERR_INVALID_VALUE;
    *result = 0.0;
    if (n == 0) return ATA_OK;
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    const size_t bytes = align256(sizeof(double) * (size_t)residual_work_elems(m, n)) + 256;
    void* buf = nullptr;
    size_t cap = 0;
    ata_status_t s = ensure(nullptr, buf, cap, bytes);
    if (s != ATA_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* out = reinterpret_cast<double*>(static_cast<unsigned char*>(buf) + bytes - 256);
    const int32_t mode = dtype == ATA_F64 ? MODE_F64 : MODE_F32;
    hipError_t e = launch_residual(mode, A, m, n, lda, C_packed, seed, static_cast<double*>(buf), out, st);
    if (e == hipSuccess) e = hipMemcpyAsync(result, out, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(buf);
    return e == hipSuccess ? ATA_OK : ATA_ERR_HIP;
}

ata_status_t ata_check_columns(ata_handle_t h, const void* A, int64_t m, int64_t n, int64_t lda,
                               ata_dtype_t dtype, const void* C_packed, const int64_t* cols, int64_t count,
                               double* result, void* stream) {
    if (!h || !result || !valid_dtype(dtype) || m < 0 || n < 0 || count < 0 || lda < std::max<int64_t>(1, n))
        return ATA_ERR_INVALID_VALUE;
    if (count > 0 && !cols) return ATA_ERR_INVALID_VALUE;
    for (int64_t k = 0; k < count; ++k)
        if (cols[k] < 0 || cols[k] >= n) return ATA_ERR_INVALID_VALUE;
    if (n > 0 && count > 0 && (!C_packed || (m > 0 && !A))) return ATA_ERR_INVALID_VALUE;
    *result = 0.0;
    if (n == 0 || count == 0) return ATA_OK;
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    const int64_t wg = ((n + 63) / 64) * ((count + 15) / 16);
    const size_t work_b = align256(sizeof(double) * (size_t)column_check_work_elems(m, n, count));
    const size_t cols_b = align256(sizeof(int64_t) * (size_t)count);
    void* buf = nullptr;
    size_t cap = 0;
    ata_status_t s = ensure(nullptr, buf, cap, work_b + cols_b);
    if (s != ATA_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* work = static_cast<double*>(buf);
    int64_t* d_cols = reinterpret_cast<int64_t*>(static_cast<unsigned char*>(buf) + work_b);
    std::vector<double> part((size_t)(2 * wg));
    const int32_t mode = dtype == ATA_F64 ? MODE_F64 : MODE_F32;
    hipError_t e = hipMemcpyAsync(d_cols, cols, sizeof(int64_t) * (size_t)count, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_column_check(mode, A, m, n, lda, C_packed, d_cols, count, work, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(part.data(), work + m * count, sizeof(double) * part.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (e != hipSuccess) return ATA_ERR_HIP;
    // workgroup sums added in workgroup order on the host (deterministic)
    double d2 = 0.0, r2 = 0.0;
    for (int64_t b = 0; b < wg; ++b) {
        d2 += part[(size_t)(2 * b)];
        r2 += part[(size_t)(2 * b + 1)];
    }
    *result = r2 > 0.0 ? std::sqrt(d2 / r2) : (d2 > 0.0 ? INFINITY : 0.0);
    return ATA_OK;
}

ata_status_t ata_gemm_tn(ata_handle_t h, const void* A, const void* B, int64_t m, int64_t n, int64_t k,
                         int64_t lda, int64_t ldb, ata_dtype_t dtype, void* C, int64_t ldc, void* stream) {
    if (!h || !valid_dtype(dtype) || m < 0 || n < 0 || k < 0 || lda < std::max<int64_t>(1, n) ||
        ldb < std::max<int64_t>(1, k) || ldc < std::max<int64_t>(1, k))
        return ATA_ERR_INVALID_VALUE;
    if (n > 0 && k > 0 && !C) return ATA_ERR_INVALID_VALUE;
    if (n > 0 && k > 0 && m > 0 && (!A || !B)) return ATA_ERR_INVALID_VALUE;
    const size_t es = dtype == ATA_F64 ? 8 : 4;
    if (n > 0 && k > 0) {
        const uintptr_t c0 = (uintptr_t)C, c1 = c0 + (size_t)((n - 1) * ldc + k) * es;
        if (m > 0) {
            const uintptr_t a0 = (uintptr_t)A, a1 = a0 + (size_t)((m - 1) * lda + n) * es;
            const uintptr_t b0 = (uintptr_t)B, b1 = b0 + (size_t)((m - 1) * ldb + k) * es;
            if ((a0 < c1 && c0 < a1) || (b0 < c1 && c0 < b1)) return ATA_ERR_INVALID_VALUE;
        }
    }
    h->report = ata_report_t{};
    h->report.flagged_nodes = -1;
    h->report.residual = -1.0;
    h->pending_flags = h->pending_residual = false;
    h->spread_plan = nullptr;
    if (n == 0 || k == 0) return ATA_OK;
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    note_capture(h, stream);
    const int32_t mode = (int32_t)dtype;
    int64_t b;
    int32_t depth, tile_cfg;
    choose(h, mode, m, std::max(n, k), b, depth, tile_cfg);
    const int64_t slots = tail_slots(h, mode, tile_cfg);
    const GemmKey key{mode, m, n, k, lda, ldb, ldc, b, depth, tile_cfg, h->split_target, h->popt.fuse_presum,
                       h->popt.variant, slots, combine_in_epilogue(h, mode, tile_cfg)};
    auto it = h->gemm_plans.find(key);
    if (it == h->gemm_plans.end()) {
        auto dp = std::make_unique<DevicePlan>();
        PlanOptions o;
        o.leaf_cutoff = b;
        o.max_depth = depth;
        o.spread_tau = 0.0;
        o.tile_cfg = tile_cfg;
        o.split_target = h->split_target;
        o.fuse_presum = h->popt.fuse_presum;
        o.variant = h->popt.variant;
        o.slots = slots;
        o.fuse_combine = key.fuse_combine;
        try {
            dp->plan = make_gemm_plan(mode, m, n, k, lda, ldb, ldc, o);
            while (dp->plan.stats.max_levels > 0 && !fits_device(h, dp->plan)) {
                o.max_depth = dp->plan.stats.max_levels - 1;
                dp->plan = make_gemm_plan(mode, m, n, k, lda, ldb, ldc, o);
            }
        } catch (const std::invalid_argument&) {
            return ATA_ERR_INVALID_VALUE;
        } catch (const std::length_error&) {
            return ATA_ERR_NOT_SUPPORTED;
        } catch (const std::exception&) {
            return ATA_ERR_INTERNAL;
        }
        const ata_status_t s = upload_plan(*dp);
        if (s != ATA_OK) return s;
        it = h->gemm_plans.emplace(key, std::move(dp)).first;
    }
    DevicePlan& dp = *it->second;
    const Plan& p = dp.plan;
    const size_t arena_bytes = (size_t)p.arena_elems * (size_t)p.elem_bytes();
    if (h->ws_limit > 0 && (int64_t)arena_bytes > h->ws_limit) return ATA_ERR_OUT_OF_MEMORY;
    const size_t old_cap = h->arena_cap;
    ata_status_t s = ensure(h, h->arena, h->arena_cap, std::max<size_t>(arena_bytes, 256));
    if (s != ATA_OK) return s;
    if (h->arena_cap != old_cap) ++h->arena_gen;
    s = ensure(h, h->aux, h->aux_cap, 512);
    if (s != ATA_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint8_t* flags = static_cast<const uint8_t*>(h->aux);     // no predicates in this plan
    BatchPtrs pq{nullptr, nullptr, reinterpret_cast<unsigned long long*>(static_cast<unsigned char*>(h->aux) + 256), 0};
    const BatchPtrs* lp = nullptr;
    if (persistent_for(h->leaf_persistent, p)) {
        pq.persistent_blocks = (int64_t)leaf_blocks_per_cu(mode, p.tile_cfg) * 256;
        lp = &pq;
    }
    hipError_t e = hipSuccess;
    hipEvent_t* ev = nullptr;
    if (take_events(h, ev) != ATA_OK) return ATA_ERR_HIP;
    auto mark = [&](int i) {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[i], st);
    };
    mark(0);
    mark(1);
    for (size_t l = 0; e == hipSuccess && l < p.presum.size(); ++l) {
        const auto& lv = p.presum[l];
        e = launch_presum(mode, dp.d_presum[l], (int)lv.size(), lv.back().elem_begin + lv.back().elems, A,
                          h->arena, flags, st, nullptr, B);
    }
    if (e == hipSuccess && !p.pack.empty())
        e = launch_pack(dp.d_pack, (int)p.pack.size(), p.pack.back().elem_begin + p.pack.back().elems, A,
                        h->arena, flags, st, nullptr, B);
    if (e == hipSuccess && !p.pack8.empty())
        e = launch_quant8(dp.d_pack8, (int)p.pack8.size(), p.pack8.back().elem_begin + p.pack8.back().elems, A,
                          h->arena, flags, st, nullptr, B);
    mark(2);
    if (e == hipSuccess) e = launch_plan_leaves(h, dp, A, C, h->arena, flags, st, lp, B);
    if (e == hipSuccess && !p.reduce.empty())
        e = launch_reduce(mode, dp.d_reduce, (int)p.reduce.size(), p.reduce.back().elem_begin + p.reduce.back().elems,
                          C, h->arena, flags, st);
    mark(3);
    for (size_t l = 0; e == hipSuccess && l < p.combine.size(); ++l) {
        const auto& lv = p.combine[l];
        if (!lv.empty())
            e = launch_combine(mode, dp.d_combine[l], (int)lv.size(), lv.back().elem_begin + lv.back().elems, C,
                               h->arena, flags, st);
    }
    mark(4);
    mark(5);
    if (e != hipSuccess) return ATA_ERR_HIP;
    fill_report(h->report, p);
    h->report.leaf_persistent = lp ? 1 : 0;
    return ATA_OK;
}

ata_status_t ata_gram_scaled(ata_handle_t h, const void* A, int64_t m, int64_t n, int64_t lda,
                             ata_dtype_t dtype, double alpha, double beta, void* C_packed, void* stream) {
    if (!h || !valid_dtype(dtype) || !std::isfinite(alpha) || !std::isfinite(beta)) return ATA_ERR_INVALID_VALUE;
    if (alpha == 1.0 && beta == 0.0) return ata_gram(h, A, m, n, lda, dtype, C_packed, stream);
    const int32_t mode = (int32_t)dtype;
    const int64_t len = n * (n + 1) / 2;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (beta == 0.0) {
        const ata_status_t s = ata_gram(h, A, m, n, lda, dtype, C_packed, stream);
        if (s != ATA_OK || n == 0) return s;
        return launch_axpby(mode, C_packed, C_packed, len, alpha, 0.0, st) == hipSuccess ? ATA_OK : ATA_ERR_HIP;
    }
    // validate against C first, so that a bad call leaves C untouched
    if (m < 0 || n < 0 || lda < std::max<int64_t>(1, n) || (n > 0 && !C_packed) || (n > 0 && m > 0 && !A))
        return ATA_ERR_INVALID_VALUE;
    if (n == 0) return ATA_OK;
    const size_t es = dtype == ATA_F64 ? 8 : 4;
    if (m > 0) {
        const uintptr_t a0 = (uintptr_t)A, a1 = a0 + (size_t)((m - 1) * lda + n) * es;
        const uintptr_t c0 = (uintptr_t)C_packed, c1 = c0 + (size_t)len * es;
        if (a0 < c1 && c0 < a1) return ATA_ERR_INVALID_VALUE;
    }
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    note_capture(h, stream);
    ata_status_t s = ensure(h, h->tmp, h->tmp_cap, (size_t)len * es);
    if (s != ATA_OK) return s;
    s = ata_gram(h, A, m, n, lda, dtype, h->tmp, stream);
    if (s != ATA_OK) return s;
    return launch_axpby(mode, h->tmp, C_packed, len, alpha, beta, st) == hipSuccess ? ATA_OK : ATA_ERR_HIP;
}

ata_status_t ata_gram_aat(ata_handle_t h, const void* A, int64_t m, int64_t n, int64_t lda,
                          ata_dtype_t dtype, void* C_packed, void* stream) {
    if (!h || !valid_dtype(dtype) || m < 0 || n < 0 || lda < std::max<int64_t>(1, n)) return ATA_ERR_INVALID_VALUE;
    if (m > 0 && !C_packed) return ATA_ERR_INVALID_VALUE;
    if (m > 0 && n > 0 && !A) return ATA_ERR_INVALID_VALUE;
    const size_t es = dtype == ATA_F64 ? 8 : 4;
    if (m > 0 && n > 0) {
        const uintptr_t a0 = (uintptr_t)A, a1 = a0 + (size_t)((m - 1) * lda + n) * es;
        const uintptr_t c0 = (uintptr_t)C_packed, c1 = c0 + (size_t)(m * (m + 1) / 2) * es;
        if (a0 < c1 && c0 < a1) return ATA_ERR_INVALID_VALUE;
    }
    if (m == 0) return ATA_OK;                     // C is 0 x 0
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    note_capture(h, stream);
    // A A^T = (A^T)^T (A^T): transpose once (one HBM pass, O(m n) against the
    // O(m^2 n) product), then the AtA plan on the n x m transpose
    ata_status_t s = ensure(h, h->tmp, h->tmp_cap, std::max<size_t>((size_t)(m * n) * es, 256));
    if (s != ATA_OK) return s;
    if (launch_transpose((int32_t)dtype, A, m, n, lda, h->tmp, static_cast<hipStream_t>(stream)) != hipSuccess)
        return ATA_ERR_HIP;
    return ata_gram(h, h->tmp, n, m, m, dtype, C_packed, stream);
}

ata_status_t ata_unpack(ata_handle_t h, const void* C_packed, int64_t n, ata_dtype_t dtype, void* C_full,
                        int64_t ldf, void* stream) {
    if (!h || !valid_dtype(dtype) || n < 0 || ldf < std::max<int64_t>(1, n)) return ATA_ERR_INVALID_VALUE;
    if (n == 0) return ATA_OK;
    if (!C_packed || !C_full) return ATA_ERR_INVALID_VALUE;
    const size_t es = dtype == ATA_F64 ? 8 : 4;
    const uintptr_t p0 = (uintptr_t)C_packed, p1 = p0 + (size_t)(n * (n + 1) / 2) * es;
    const uintptr_t f0 = (uintptr_t)C_full, f1 = f0 + (size_t)((n - 1) * ldf + n) * es;
    if (p0 < f1 && f0 < p1) return ATA_ERR_INVALID_VALUE;
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    return launch_unpack((int32_t)dtype, C_packed, n, C_full, ldf, static_cast<hipStream_t>(stream)) == hipSuccess
               ? ATA_OK : ATA_ERR_HIP;
}

namespace {

// Enqueue every phase of a merged batch plan on `st` (also used for capture).
// `ev`: six phase events of an eager profiled call, or null.
hipError_t enqueue_batch(ata_ctx* h, BatchEntry& be, hipStream_t st, hipEvent_t* ev = nullptr) {
    const Plan& p = be.dp->plan;
    DevicePlan& dp = *be.dp;
    const int32_t mode = p.mode;
    hipError_t e = hipSuccess;
    auto mark = [&](int i) {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[i], st);
    };
    mark(0);
    e = hipMemcpyAsync(be.d_A, be.pinned, sizeof(void*) * 2 * (size_t)be.nprob, hipMemcpyHostToDevice, st);
    const int64_t slots = (int64_t)leaf_blocks_per_cu(mode, p.tile_cfg) * 256;
    BatchPtrs bp{be.d_A, be.d_C, persistent_for(h->batch_persistent, p) ? be.d_counter : nullptr, slots};
    BatchPtrs bq{be.d_A, be.d_C, nullptr, 0};
    const int32_t q0 = p.pack8_norm;
    if (e == hipSuccess && p.fallback) {
        const ColDesc& l1 = be.col1.back();
        const ColDesc& l2 = be.col2.back();
        if (q0 > 0)
            e = launch_quant8(dp.d_pack8, q0, p.pack8[q0 - 1].elem_begin + p.pack8[q0 - 1].elems, nullptr, h->arena,
                              be.d_flags, st, &bq, nullptr, be.d_partial);
        if (e == hipSuccess)
            e = launch_colnorms(be.d_col1, (int)be.col1.size(), l1.elem_begin + l1.elems, be.d_col2,
                                (int)be.col2.size(), l2.elem_begin + l2.elems, nullptr, be.d_A, be.d_partial,
                                be.d_nu, st, h->arena, has_pack(be.col1));
        if (e == hipSuccess)
            e = launch_flags(be.d_nu, dp.d_nodes, (int)p.nodes.size(),
                             h->popt.spread_tau * h->popt.spread_tau, be.d_flags, st);
    }
    mark(1);
    for (size_t l = 0; e == hipSuccess && l < p.presum.size(); ++l) {
        const auto& lv = p.presum[l];
        if (!lv.empty())
            e = launch_presum(mode, dp.d_presum[l], (int)lv.size(), lv.back().elem_begin + lv.back().elems,
                              nullptr, h->arena, be.d_flags, st, &bq);
    }
    if (e == hipSuccess && !p.pack.empty())
        e = launch_pack(dp.d_pack, (int)p.pack.size(), p.pack.back().elem_begin + p.pack.back().elems,
                        nullptr, h->arena, be.d_flags, st, &bq);
    if (e == hipSuccess && (int32_t)p.pack8.size() > q0)
        e = launch_quant8(dp.d_pack8 + q0, (int)p.pack8.size() - q0, p.pack8.back().elem_begin + p.pack8.back().elems,
                          nullptr, h->arena, be.d_flags, st, &bq);
    mark(2);
    if (e == hipSuccess)
        e = launch_leaves(mode, p.tile_cfg, dp.d_leaves, (int)p.leaves.size(), p.total_tiles, nullptr,
                          nullptr, h->arena, be.d_flags, h->chunk, h->band, st, &bp);
    if (e == hipSuccess && !p.fb_leaves.empty())
        e = launch_fallback_leaves(dp.d_fb_leaves, (int)p.fb_leaves.size(), p.fb_tiles, nullptr, nullptr,
                                   h->arena, be.d_flags, h->chunk, h->band, st, &bq);
    if (e == hipSuccess && !p.reduce.empty())
        e = launch_reduce(mode, dp.d_reduce, (int)p.reduce.size(), p.reduce.back().elem_begin + p.reduce.back().elems,
                          nullptr, h->arena, be.d_flags, st, &bq);
    mark(3);
    for (size_t l = 0; e == hipSuccess && l < p.combine.size(); ++l) {
        const auto& lv = p.combine[l];
        if (!lv.empty())
            e = launch_combine(mode, dp.d_combine[l], (int)lv.size(), lv.back().elem_begin + lv.back().elems,
                               nullptr, h->arena, be.d_flags, st, &bq);
    }
    mark(4);
    mark(5);
    return e;
}

}  // namespace

ata_status_t ata_gram_batched(ata_handle_t h, int64_t batch, const void* const* A,
                              const int64_t* m, const int64_t* n, const int64_t* lda,
                              ata_dtype_t dtype, void* const* C_packed, void* stream) {
    if (!h || batch <= 0 || !A || !m || !n || !lda || !C_packed || !valid_dtype(dtype))
        return ATA_ERR_INVALID_VALUE;
    const size_t es = dtype == ATA_F64 ? 8 : 4;
    for (int64_t i = 0; i < batch; ++i) {
        bool bad = m[i] < 0 || n[i] < 0 || lda[i] < std::max<int64_t>(1, n[i]) ||
                   (n[i] > 0 && !C_packed[i]) || (n[i] > 0 && m[i] > 0 && !A[i]);
        if (!bad && n[i] > 0 && m[i] > 0) {
            const uintptr_t a0 = (uintptr_t)A[i], a1 = a0 + (size_t)((m[i] - 1) * lda[i] + n[i]) * es;
            const uintptr_t c0 = (uintptr_t)C_packed[i], c1 = c0 + (size_t)(n[i] * (n[i] + 1) / 2) * es;
            bad = a0 < c1 && c0 < a1;
        }
        if (bad) {
            h->report = ata_report_t{};
            h->report.m = -(i + 1);
            h->report.flagged_nodes = -1;
            h->report.residual = -1.0;
            return ATA_ERR_INVALID_VALUE;
        }
    }
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    note_capture(h, stream);
    h->spread_plan = nullptr;
    const int32_t mode = (int32_t)dtype;
    const bool fb = mode != MODE_F64 && h->popt.spread_tau > 0;
    // the batch runs one leaf kernel, so one tile shape: the handle's, or the
    // batch autotuner's for this signature when the options are defaults
    int32_t tile_cfg = tiled_mode(mode) && h->popt.tile_cfg > 0 ? h->popt.tile_cfg : 0;
    const ata_tune_entry_t* bt = nullptr;
    if (h->popt.leaf_cutoff <= 0 && h->popt.max_depth < 0 && !h->batch_tune.empty()) {
        auto f = h->batch_tune.find(batch_signature(mode, batch, m, n, lda));
        if (f != h->batch_tune.end()) {
            bt = &f->second;
            if (tiled_mode(mode)) tile_cfg = bt->leaf_tile;
        }
    }
    std::vector<int64_t> bs((size_t)batch);
    std::vector<int32_t> ds((size_t)batch);
    const int64_t slots = tail_slots(h, mode, tile_cfg);
    BatchKey key{mode, h->popt.leaf_cutoff, h->popt.max_depth, fb, tile_cfg, h->split_target, h->popt.fuse_presum,
                 h->popt.variant, slots, {}};
    key.shapes.reserve(5 * (size_t)batch);
    for (int64_t i = 0; i < batch; ++i) {
        int32_t tile_i;
        choose(h, mode, m[i], n[i], bs[(size_t)i], ds[(size_t)i], tile_i, h->batch_use_table);
        if (bt) {
            bs[(size_t)i] = bt->leaf_cutoff;
            ds[(size_t)i] = bt->max_depth;
        }
        key.shapes.push_back(m[i]);
        key.shapes.push_back(n[i]);
        key.shapes.push_back(lda[i]);
        key.shapes.push_back(bs[(size_t)i]);
        key.shapes.push_back(ds[(size_t)i]);
    }
    auto it = h->batches.find(key);
    if (it == h->batches.end()) {
        auto be = std::make_unique<BatchEntry>();
        be->nprob = batch;
        std::vector<Plan> parts;
        parts.reserve((size_t)batch);
        try {
            for (int64_t i = 0; i < batch; ++i) {
                PlanOptions o;
                o.leaf_cutoff = bs[(size_t)i];
                o.max_depth = ds[(size_t)i];
                o.spread_tau = fb ? h->popt.spread_tau : 0.0;
                o.tile_cfg = tile_cfg;
                o.split_target = 0;          // the merged plan is split as a whole
                o.fuse_presum = h->popt.fuse_presum;
                o.variant = h->popt.variant;
                parts.push_back(make_plan(mode, m[i], n[i], lda[i], o));
            }
            be->dp = std::make_unique<DevicePlan>();
            be->dp->plan = merge_plans(parts, h->split_target, slots);
        } catch (const std::invalid_argument&) {
            return ATA_ERR_INVALID_VALUE;
        } catch (const std::length_error&) {
            return ATA_ERR_NOT_SUPPORTED;
        } catch (const std::exception&) {
            return ATA_ERR_INTERNAL;
        }
        const Plan& mp = be->dp->plan;
        // column-norm tasks (every problem, so the merged norm array is
        // complete); split-BF16 members' A packing moves into pass 1
        int64_t part_off = 0, nu_off = 0;
        if (mp.fallback) {
            build_colnorm_tasks(m, n, lda, batch, be->col1, be->col2, &part_off);
            fuse_pack_into_norms(be->dp->plan, be->col1);
            fuse_norms_into_quant(be->dp->plan, be->col1, be->col2, part_off);
            for (int64_t i = 0; i < batch; ++i) nu_off += n[i];
        }
        ata_status_t st0 = upload_plan(*be->dp);
        if (st0 != ATA_OK) return st0;
        // auxiliary device buffer owned by the batch entry
        const size_t ptr_b = align256(sizeof(void*) * 2 * (size_t)batch);
        const size_t cnt_b = 256;
        const size_t flg_b = align256(std::max<size_t>(mp.nodes.size(), 1));
        const size_t par_b = align256(sizeof(double) * (size_t)std::max<int64_t>(part_off, 1));
        const size_t nu_b = align256(sizeof(double) * (size_t)std::max<int64_t>(nu_off, 1));
        const size_t c1_b = align256(sizeof(ColDesc) * be->col1.size());
        const size_t c2_b = align256(sizeof(ColDesc) * be->col2.size());
        be->aux_bytes = ptr_b + cnt_b + flg_b + par_b + nu_b + c1_b + c2_b;
        if (hipMalloc(&be->aux, be->aux_bytes) != hipSuccess) {
            be->aux = nullptr;
            return ATA_ERR_OUT_OF_MEMORY;
        }
        unsigned char* a = static_cast<unsigned char*>(be->aux);
        be->d_A = reinterpret_cast<const void**>(a);
        be->d_C = reinterpret_cast<void**>(a) + batch;
        be->d_counter = reinterpret_cast<unsigned long long*>(a + ptr_b);
        be->d_flags = a + ptr_b + cnt_b;
        be->d_partial = reinterpret_cast<double*>(a + ptr_b + cnt_b + flg_b);
        be->d_nu = reinterpret_cast<double*>(a + ptr_b + cnt_b + flg_b + par_b);
        be->d_col1 = reinterpret_cast<ColDesc*>(a + ptr_b + cnt_b + flg_b + par_b + nu_b);
        be->d_col2 = reinterpret_cast<ColDesc*>(a + ptr_b + cnt_b + flg_b + par_b + nu_b + c1_b);
        if (!be->col1.empty()) {
            if (hipMemcpy(be->d_col1, be->col1.data(), sizeof(ColDesc) * be->col1.size(), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(be->d_col2, be->col2.data(), sizeof(ColDesc) * be->col2.size(), hipMemcpyHostToDevice) != hipSuccess)
                return ATA_ERR_HIP;
        }
        if (hipHostMalloc(reinterpret_cast<void**>(&be->pinned), sizeof(void*) * 2 * (size_t)batch, 0) != hipSuccess) {
            be->pinned = nullptr;
            return ATA_ERR_OUT_OF_MEMORY;
        }
        if (hipEventCreateWithFlags(&be->done, hipEventDisableTiming) != hipSuccess) return ATA_ERR_HIP;
        it = h->batches.emplace(key, std::move(be)).first;
    }
    BatchEntry& be = *it->second;
    const Plan& mp = be.dp->plan;
    const size_t arena_bytes = (size_t)mp.arena_elems * (size_t)mp.elem_bytes();
    if (h->ws_limit > 0 && (int64_t)(arena_bytes + be.aux_bytes) > h->ws_limit) return ATA_ERR_OUT_OF_MEMORY;
    const size_t old_cap = h->arena_cap;
    ata_status_t s = ensure(h, h->arena, h->arena_cap, std::max<size_t>(arena_bytes, 256));
    if (s != ATA_OK) return s;
    if (h->arena_cap != old_cap) ++h->arena_gen;
    // stage the pointers; a previous replay may still be copying them
    bool changed = !be.launched;
    for (int64_t i = 0; i < batch && !changed; ++i)
        changed = be.pinned[i] != A[i] || be.pinned[batch + i] != C_packed[i];
    if (changed) {
        if (be.launched && hipEventSynchronize(be.done) != hipSuccess) return ATA_ERR_HIP;
        for (int64_t i = 0; i < batch; ++i) {
            be.pinned[i] = const_cast<void*>(A[i]);
            be.pinned[batch + i] = C_packed[i];
        }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (!h->batch_graph) {
        hipEvent_t* ev = nullptr;
        if (take_events(h, ev) != ATA_OK) return ATA_ERR_HIP;
        e = enqueue_batch(h, be, st, ev);
        if (e == hipSuccess) e = hipEventRecord(be.done, st);
    } else {
        if (!h->batch_stream) {
            if (hipStreamCreateWithFlags(&h->batch_stream, hipStreamNonBlocking) != hipSuccess) return ATA_ERR_HIP;
            if (hipEventCreateWithFlags(&h->batch_in, hipEventDisableTiming) != hipSuccess) return ATA_ERR_HIP;
        }
        if (!be.exec || be.arena_gen != h->arena_gen || be.graph_persistent != persistent_for(h->batch_persistent, be.dp->plan)) {
            if (be.exec) {
                if (be.launched && hipEventSynchronize(be.done) != hipSuccess) return ATA_ERR_HIP;
                (void)hipGraphExecDestroy(be.exec);
                (void)hipGraphDestroy(be.graph);
                be.exec = nullptr;
                be.graph = nullptr;
            }
            (void)leaf_blocks_per_cu(mode, mp.tile_cfg);   // occupancy query outside the capture
            e = hipStreamBeginCapture(h->batch_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t e1 = enqueue_batch(h, be, h->batch_stream);
                e = hipStreamEndCapture(h->batch_stream, &be.graph);
                if (e1 != hipSuccess) e = e1;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&be.exec, be.graph, nullptr, nullptr, 0);
            if (e != hipSuccess) return ATA_ERR_HIP;
            be.arena_gen = h->arena_gen;
            be.graph_persistent = persistent_for(h->batch_persistent, be.dp->plan);
        }
        e = hipEventRecord(h->batch_in, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->batch_stream, h->batch_in, 0);
        if (e == hipSuccess) e = hipGraphLaunch(be.exec, h->batch_stream);
        if (e == hipSuccess) e = hipEventRecord(be.done, h->batch_stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, be.done, 0);
    }
    if (e != hipSuccess) return ATA_ERR_HIP;
    be.launched = true;
    fill_report(h->report, mp);
    h->report.leaf_persistent = persistent_for(h->batch_persistent, mp) ? 1 : 0;
    h->report.m = 0;
    h->report.n = 0;
    h->report.lda = 0;
    h->pending_flags = false;
    h->pending_residual = false;
    return ATA_OK;
}

ata_status_t ata_autotune(ata_handle_t h, const void* A, int64_t m, int64_t n, int64_t lda,
                          ata_dtype_t dtype, void* C_packed, void* stream, ata_tune_entry_t* best) {
    if (!h || !valid_dtype(dtype) || m <= 0 || n <= 0 || lda < n || !A || !C_packed)
        return ATA_ERR_INVALID_VALUE;
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    const int32_t mode = (int32_t)dtype;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const PlanOptions saved = h->popt;
    const bool saved_profile = h->profile;
    h->profile = false;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return ATA_ERR_HIP;
    ata_tune_entry_t top{0, 0, 0, 1e30};
    std::vector<ata_tune_entry_t> all;            // first pass: every candidate once
    std::vector<int64_t> cutoffs;
    for (int64_t b = 128; ; b *= 2) {
        cutoffs.push_back(b);
        if (b >= n) break;
    }
    const int32_t dmax = std::min<int32_t>(default_max_depth(mode, m), 3);
    // mean ms of `reps` back-to-back calls with the handle's current options
    auto time_calls = [&](int reps, double& per) -> ata_status_t {
        if (hipEventRecord(e0, st) != hipSuccess) return ATA_ERR_HIP;
        for (int r = 0; r < reps; ++r) {
            const ata_status_t q = ata_gram(h, A, m, n, lda, dtype, C_packed, stream);
            if (q != ATA_OK) return q;
        }
        float ms = 0.f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return ATA_ERR_HIP;
        per = ms / reps;
        return ATA_OK;
    };
    const std::vector<int32_t> tiles = tile_candidates(mode);
    ata_status_t rs = ATA_OK;
    for (int64_t b : cutoffs) {
        for (int32_t d = 0; d <= dmax; ++d) {
            if (b >= n && d > 0) break;            // a single leaf: depth does not matter
            for (const int32_t tl : tiles) {
                h->popt.leaf_cutoff = b;
                h->popt.max_depth = d;
                h->popt.tile_cfg = tl;
                // skip depth caps the recursion cannot reach
                Plan probe;
                try {
                    PlanOptions o;
                    o.leaf_cutoff = b;
                    o.max_depth = d;
                    o.spread_tau = 0.0;
                    probe = make_plan(mode, m, n, lda, o);
                } catch (const std::exception&) {
                    continue;
                }
                if (d > 0 && probe.stats.max_levels < d) continue;
                rs = ata_gram(h, A, m, n, lda, dtype, C_packed, stream);   // warm-up (plans, arena)
                if (rs == ATA_ERR_NOT_SUPPORTED || rs == ATA_ERR_OUT_OF_MEMORY) {
                    rs = ATA_OK;                    // this candidate cannot run here: skip it
                    continue;
                }
                if (rs != ATA_OK) break;
                double per = 0.0;
                rs = time_calls(3, per);
                if (rs != ATA_OK) break;
                all.push_back(ata_tune_entry_t{b, d, tl, per});
            }
            if (rs != ATA_OK) break;
        }
        if (rs != ATA_OK) break;
    }
    // second pass: the four fastest again, interleaved over three rounds of
    // five calls each; a candidate scores its best round (a single pass is
    // at the mercy of clock and power transients)
    if (rs == ATA_OK && !all.empty()) {
        std::stable_sort(all.begin(), all.end(),
                         [](const ata_tune_entry_t& x, const ata_tune_entry_t& y) { return x.ms < y.ms; });
        if (all.size() > 4) all.resize(4);
        std::vector<double> score(all.size(), 1e30);
        for (int round = 0; round < 3 && rs == ATA_OK; ++round) {
            for (size_t c = 0; c < all.size() && rs == ATA_OK; ++c) {
                h->popt.leaf_cutoff = all[c].leaf_cutoff;
                h->popt.max_depth = all[c].max_depth;
                h->popt.tile_cfg = all[c].leaf_tile;
                rs = ata_gram(h, A, m, n, lda, dtype, C_packed, stream);
                double per = 0.0;
                if (rs == ATA_OK) rs = time_calls(5, per);
                if (rs == ATA_OK) score[c] = std::min(score[c], per);
            }
        }
        for (size_t c = 0; c < all.size(); ++c)
            if (score[c] < top.ms) top = ata_tune_entry_t{all[c].leaf_cutoff, all[c].max_depth, all[c].leaf_tile, score[c]};
    }
    h->popt = saved;
    h->profile = saved_profile;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rs != ATA_OK) return rs;
    h->tune[TuneKey{mode, bucket(m), bucket(n)}] = top;
    if (best) *best = top;
    return ATA_OK;
}

ata_status_t ata_autotune_batched(ata_handle_t h, int64_t batch, const void* const* A, const int64_t* m,
                                  const int64_t* n, const int64_t* lda, ata_dtype_t dtype,
                                  void* const* C_packed, void* stream, ata_tune_entry_t* best) {
    if (!h || batch <= 0 || !m || !n || !lda || !valid_dtype(dtype)) return ATA_ERR_INVALID_VALUE;
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    const int32_t mode = (int32_t)dtype;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const PlanOptions saved = h->popt;
    const bool saved_profile = h->profile;
    h->profile = false;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return ATA_ERR_HIP;
    ata_tune_entry_t top{0, 0, 0, 1e30};
    const std::vector<int32_t> tiles = tile_candidates(mode);
    int64_t mmax = 0;
    for (int64_t i = 0; i < batch; ++i) mmax = std::max(mmax, m[i]);
    const int32_t dmax = std::min<int32_t>(default_max_depth(mode, mmax), 2);
    ata_status_t rs = ATA_OK;
    for (int64_t b = 128; b <= 4096 && rs == ATA_OK; b *= 2) {
        for (int32_t d = 0; d <= dmax && rs == ATA_OK; ++d) {
            for (const int32_t tl : tiles) {
                h->popt.leaf_cutoff = b;
                h->popt.max_depth = d;
                h->popt.tile_cfg = tl;
                rs = ata_gram_batched(h, batch, A, m, n, lda, dtype, C_packed, stream);   // plan + graph
                if (rs == ATA_ERR_NOT_SUPPORTED || rs == ATA_ERR_OUT_OF_MEMORY) {
                    rs = ATA_OK;
                    continue;
                }
                if (rs != ATA_OK) break;
                const int reps = 3;
                if (hipEventRecord(e0, st) != hipSuccess) { rs = ATA_ERR_HIP; break; }
                for (int r = 0; r < reps && rs == ATA_OK; ++r)
                    rs = ata_gram_batched(h, batch, A, m, n, lda, dtype, C_packed, stream);
                if (rs != ATA_OK) break;
                float ms = 0.f;
                if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rs = ATA_ERR_HIP; break; }
                const double per = ms / reps;
                if (per < top.ms) top = ata_tune_entry_t{b, d, tl, per};
            }
        }
    }
    h->popt = saved;
    h->profile = saved_profile;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rs != ATA_OK) return rs;
    if (top.leaf_cutoff == 0) return ATA_ERR_NOT_SUPPORTED;
    h->batch_tune[batch_signature(mode, batch, m, n, lda)] = top;
    if (best) *best = top;
    return ATA_OK;
}

ata_status_t ata_tune_save(ata_handle_t h, const char* path) {
    if (!h || !path) return ATA_ERR_INVALID_VALUE;
    std::ofstream f(path);
    if (!f) return ATA_ERR_INVALID_VALUE;
    f << "[\n";
    size_t i = 0;
    for (const auto& kv : h->tune) {
        f << "  {\"arch\": \"" << h->arch << "\", \"dtype\": " << kv.first.mode << ", \"m_bucket\": "
          << kv.first.mb << ", \"n_bucket\": " << kv.first.nb << ", \"leaf_cutoff\": " << kv.second.leaf_cutoff
          << ", \"max_depth\": " << kv.second.max_depth << ", \"leaf_tile\": " << kv.second.leaf_tile
          << ", \"ms\": " << kv.second.ms << "}" << (++i < h->tune.size() ? "," : "") << "\n";
    }
    f << "]\n";
    return f ? ATA_OK : ATA_ERR_INTERNAL;
}

ata_status_t ata_tune_load(ata_handle_t h, const char* path) {
    if (!h || !path) return ATA_ERR_INVALID_VALUE;
    std::ifstream f(path);
    if (!f) return ATA_ERR_INVALID_VALUE;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    auto num = [&](const std::string& obj, const char* key, double& out) {
        const std::string k = std::string("\"") + key + "\":";
        const size_t p = obj.find(k);
        if (p == std::string::npos) return false;
        out = std::strtod(obj.c_str() + p + k.size(), nullptr);
        return true;
    };
    size_t pos = 0;
    while ((pos = text.find('{', pos)) != std::string::npos) {
        const size_t end = text.find('}', pos);
        if (end == std::string::npos) break;
        const std::string obj = text.substr(pos, end - pos + 1);
        pos = end + 1;
        const size_t a = obj.find("\"arch\": \"");
        if (a == std::string::npos) continue;
        const size_t a0 = a + 9, a1 = obj.find('"', a0);
        if (obj.substr(a0, a1 - a0) != h->arch) continue;
        double dt, mb, nb, b, d, tl, ms;
        if (!num(obj, "dtype", dt) || !num(obj, "m_bucket", mb) || !num(obj, "n_bucket", nb) ||
            !num(obj, "leaf_cutoff", b) || !num(obj, "max_depth", d) || !num(obj, "leaf_tile", tl) ||
            !num(obj, "ms", ms))
            continue;
        h->tune[TuneKey{(int32_t)dt, (int32_t)mb, (int32_t)nb}] =
            ata_tune_entry_t{(int64_t)b, (int32_t)d, (int32_t)tl, ms};
    }
    return ATA_OK;
}

ata_status_t ata_get_spread(ata_handle_t h, double* nu, int64_t n, int64_t* node_c0, int64_t* node_w,
                            uint8_t* flags, int64_t cap, int64_t* count) {
    if (!h || n < 0 || cap < 0) return ATA_ERR_INVALID_VALUE;
    if (!h->spread_plan) return ATA_ERR_INVALID_VALUE;
    const Plan& p = h->spread_plan->plan;
    if (nu && n != p.n) return ATA_ERR_INVALID_VALUE;
    const int64_t nodes = (int64_t)p.nodes.size();
    if (count) *count = nodes;
    const int64_t k = std::min(cap, nodes);
    for (int64_t i = 0; i < k; ++i) {
        if (node_c0) node_c0[i] = p.nodes[(size_t)i].c0;
        if (node_w) node_w[i] = p.nodes[(size_t)i].w;
    }
    if (!nu && !(flags && k > 0)) return ATA_OK;
    if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
    if (hipStreamSynchronize(h->spread_stream) != hipSuccess) return ATA_ERR_HIP;
    if (nu && n > 0 && hipMemcpy(nu, h->spread_nu, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess)
        return ATA_ERR_HIP;
    if (flags && k > 0 && hipMemcpy(flags, h->spread_flags, (size_t)k, hipMemcpyDeviceToHost) != hipSuccess)
        return ATA_ERR_HIP;
    return ATA_OK;
}

ata_status_t ata_get_report(ata_handle_t h, ata_report_t* out) {
    if (!h || !out) return ATA_ERR_INVALID_VALUE;
    if (h->events_used) {
        if (hipSetDevice(h->device) != hipSuccess || drain_events(h) != hipSuccess) return ATA_ERR_HIP;
    }
    h->report.profiled_calls = h->profiled_calls;
    for (int i = 0; i < 5; ++i) h->report.phase_ms[i] = h->phase_ms[i];
    if (h->pending_flags || h->pending_residual) {
        if (hipSetDevice(h->device) != hipSuccess) return ATA_ERR_HIP;
        if (hipStreamSynchronize(h->last_stream) != hipSuccess) return ATA_ERR_HIP;
        if (h->pending_flags) {
            std::vector<uint8_t> f((size_t)h->last_nodes);
            if (hipMemcpy(f.data(), h->last_flags, f.size(), hipMemcpyDeviceToHost) != hipSuccess)
                return ATA_ERR_HIP;
            h->report.flagged_nodes = (int64_t)std::count(f.begin(), f.end(), (uint8_t)1);
        }
        if (h->pending_residual) {
            double r = -1.0;
            if (hipMemcpy(&r, h->last_residual, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
                return ATA_ERR_HIP;
            h->report.residual = r;
        }
        h->pending_flags = h->pending_residual = false;
    }
    *out = h->report;
    return ATA_OK;
}

}  // extern "C"
