// C ABI of the library (declared in include/ata.h): argument validation,
// plan cache, workspace, and the launch sequence of one Gram product.
#include "ata.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
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
    bool operator<(const PlanKey& o) const {
        return std::tie(mode, m, n, lda, b, depth, fb, tile_cfg) <
               std::tie(o.mode, o.m, o.n, o.lda, o.b, o.depth, o.fb, o.tile_cfg);
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
    std::vector<CombineDesc*> d_combine;
    NodeDesc* d_nodes = nullptr;
    ~DevicePlan() { if (d_buf) (void)hipFree(d_buf); }
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct ata_ctx {
    int device = 0;
    PlanOptions popt;
    bool residual = false;
    uint64_t seed = 0x5EEDull;
    int64_t ws_limit = 0;
    int chunk = 16;
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
    // phase profiling: six events per profiled call, summed at report time
    bool profile = false;
    std::vector<hipEvent_t> events;   // pool, grows on demand
    size_t events_used = 0;
    int64_t profiled_calls = 0;
    double phase_ms[5] = {0, 0, 0, 0, 0};
};

namespace {

ata_status_t hip_status(hipError_t e) { return e == hipSuccess ? ATA_OK : ATA_ERR_HIP; }

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

ata_status_t ensure(void*& ptr, size_t& cap, size_t bytes) {
    if (bytes <= cap) return ATA_OK;
    if (ptr) {
        // hipFree waits for outstanding work on the device
        if (hipFree(ptr) != hipSuccess) return ATA_ERR_HIP;
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

ata_status_t upload_plan(DevicePlan& dp) {
    const Plan& p = dp.plan;
    size_t bytes = align256(p.leaves.size() * sizeof(LeafDesc));
    for (auto& l : p.presum) bytes += align256(l.size() * sizeof(PresumDesc));
    for (auto& l : p.combine) bytes += align256(l.size() * sizeof(CombineDesc));
    bytes += align256(p.nodes.size() * sizeof(NodeDesc));
    bytes += align256(p.pack.size() * sizeof(PackDesc));
    bytes += align256(p.fb_leaves.size() * sizeof(LeafDesc));
    if (bytes == 0) return ATA_OK;
    std::vector<unsigned char> host(bytes, 0);
    if (hipMalloc(&dp.d_buf, bytes) != hipSuccess) {
        dp.d_buf = nullptr;
        return ATA_ERR_OUT_OF_MEMORY;
    }
    size_t off = 0;
    auto put = [&](const void* src, size_t n) {
        std::memcpy(host.data() + off, src, n);
        void* d = static_cast<unsigned char*>(dp.d_buf) + off;
        off += align256(n);
        return d;
    };
    dp.d_leaves = static_cast<LeafDesc*>(put(p.leaves.data(), p.leaves.size() * sizeof(LeafDesc)));
    for (auto& l : p.presum) dp.d_presum.push_back(static_cast<PresumDesc*>(put(l.data(), l.size() * sizeof(PresumDesc))));
    for (auto& l : p.combine) dp.d_combine.push_back(static_cast<CombineDesc*>(put(l.data(), l.size() * sizeof(CombineDesc))));
    dp.d_nodes = static_cast<NodeDesc*>(put(p.nodes.data(), p.nodes.size() * sizeof(NodeDesc)));
    dp.d_pack = static_cast<PackDesc*>(put(p.pack.data(), p.pack.size() * sizeof(PackDesc)));
    dp.d_fb_leaves = static_cast<LeafDesc*>(put(p.fb_leaves.data(), p.fb_leaves.size() * sizeof(LeafDesc)));
    return hip_status(hipMemcpy(dp.d_buf, host.data(), bytes, hipMemcpyHostToDevice));
}

bool valid_dtype(int d) { return d >= ATA_F64 && d <= ATA_F32_FP8E4M3; }

// Bytes of auxiliary device memory one call needs (flags, norms, residual).
struct AuxLayout {
    size_t flags_off = 0, part_off = 0, nu_off = 0, res_work_off = 0, res_off = 0, total = 0;
};

AuxLayout aux_layout(const Plan& p, bool residual) {
    AuxLayout a;
    size_t off = 0;
    a.flags_off = off;
    off += align256(std::max<size_t>(p.nodes.size(), 1));
    a.part_off = off;
    off += align256(sizeof(double) * (size_t)(p.fallback ? colnorm_chunks(p.m, p.n) * p.n : 0));
    a.nu_off = off;
    off += align256(sizeof(double) * (size_t)(p.fallback ? p.n : 0));
    a.res_work_off = off;
    off += align256(sizeof(double) * (size_t)(residual ? residual_work_elems(p.m, p.n) : 0));
    a.res_off = off;
    off += align256(sizeof(double));
    a.total = off;
    return a;
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
    *out = h;
    return ATA_OK;
}

ata_status_t ata_destroy(ata_handle_t h) {
    if (!h) return ATA_OK;
    (void)hipSetDevice(h->device);
    h->plans.clear();
    (void)hipDeviceSynchronize();
    clear_events(h);
    if (h->arena) (void)hipFree(h->arena);
    if (h->aux) (void)hipFree(h->aux);
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
            if (value != 0 && value != 1 && value != 2) return ATA_ERR_INVALID_VALUE;
            h->popt.tile_cfg = (int32_t)value;
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
    if (dtype == ATA_F32_FP8E4M3) return ATA_ERR_NOT_SUPPORTED;
    PlanOptions o;
    o.leaf_cutoff = leaf_cutoff > 0 ? leaf_cutoff : 0;
    o.max_depth = max_depth;
    o.spread_tau = 0.0;
    Plan p;
    try {
        p = make_plan((int32_t)dtype, m, n, std::max<int64_t>(1, n), o);
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
    }
    return ATA_OK;
}

ata_status_t ata_gram(ata_handle_t h, const void* A, int64_t m, int64_t n, int64_t lda,
                      ata_dtype_t dtype, void* C_packed, void* stream) {
    if (!h || !valid_dtype(dtype) || m < 0 || n < 0 || lda < std::max<int64_t>(1, n))
        return ATA_ERR_INVALID_VALUE;
    if (n > 0 && !C_packed) return ATA_ERR_INVALID_VALUE;
    if (n > 0 && m > 0 && !A) return ATA_ERR_INVALID_VALUE;
    if (dtype == ATA_F32_FP8E4M3) return ATA_ERR_NOT_SUPPORTED;
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
    const int32_t mode = (int32_t)dtype;
    const int64_t b = h->popt.leaf_cutoff > 0 ? h->popt.leaf_cutoff : default_leaf_cutoff(mode, m, n);
    const int32_t depth = h->popt.max_depth >= 0 ? h->popt.max_depth : default_max_depth(mode);
    const bool fb = mode != MODE_F64 && h->popt.spread_tau > 0 && m > 0;
    const int32_t tile_cfg = mode == MODE_BF16X3 ? h->popt.tile_cfg : 0;
    const PlanKey key{mode, m, n, lda, b, depth, fb, tile_cfg};
    auto it = h->plans.find(key);
    if (it == h->plans.end()) {
        auto dp = std::make_unique<DevicePlan>();
        PlanOptions o;
        o.leaf_cutoff = b;
        o.max_depth = depth;
        o.spread_tau = fb ? h->popt.spread_tau : 0.0;
        o.tile_cfg = tile_cfg;
        try {
            dp->plan = make_plan(mode, m, n, lda, o);
        } catch (const std::invalid_argument&) {
            return ATA_ERR_INVALID_VALUE;
        } catch (const std::exception&) {
            return ATA_ERR_INTERNAL;
        }
        const ata_status_t s = upload_plan(*dp);
        if (s != ATA_OK) return s;
        it = h->plans.emplace(key, std::move(dp)).first;
    }
    DevicePlan& dp = *it->second;
    const Plan& p = dp.plan;
    const AuxLayout ax = aux_layout(p, h->residual);
    const size_t arena_bytes = (size_t)p.arena_elems * (size_t)p.elem_bytes();
    if (h->ws_limit > 0 && (int64_t)(arena_bytes + ax.total) > h->ws_limit) return ATA_ERR_OUT_OF_MEMORY;
    ata_status_t s = ensure(h->arena, h->arena_cap, std::max<size_t>(arena_bytes, 256));
    if (s != ATA_OK) return s;
    s = ensure(h->aux, h->aux_cap, ax.total);
    if (s != ATA_OK) return s;

    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char* aux = static_cast<unsigned char*>(h->aux);
    uint8_t* flags = aux + ax.flags_off;
    double* partial = reinterpret_cast<double*>(aux + ax.part_off);
    double* nu = reinterpret_cast<double*>(aux + ax.nu_off);
    double* res_work = reinterpret_cast<double*>(aux + ax.res_work_off);
    double* res = reinterpret_cast<double*>(aux + ax.res_off);
    hipError_t e = hipSuccess;
    hipEvent_t* ev = nullptr;
    if (h->profile) {
        if (h->events_used + EVENTS_PER_CALL > 4096) {
            e = drain_events(h);
            if (e != hipSuccess) return ATA_ERR_HIP;
        }
        while (h->events.size() < h->events_used + EVENTS_PER_CALL) {
            hipEvent_t x;
            if (hipEventCreate(&x) != hipSuccess) return ATA_ERR_HIP;
            h->events.push_back(x);
        }
        ev = h->events.data() + h->events_used;
        h->events_used += EVENTS_PER_CALL;
    }
    auto mark = [&](int i) {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[i], st);
    };
    mark(0);
    if (p.fallback) {
        e = launch_colnorms(static_cast<const float*>(A), m, n, lda, partial, colnorm_chunks(m, n), nu, st);
        if (e == hipSuccess)
            e = launch_flags(nu, dp.d_nodes, (int)p.nodes.size(), h->popt.spread_tau * h->popt.spread_tau, flags, st);
    }
    mark(1);
    for (size_t l = 0; e == hipSuccess && l < p.presum.size(); ++l) {
        const auto& lv = p.presum[l];
        e = launch_presum(mode, dp.d_presum[l], (int)lv.size(), lv.back().elem_begin + lv.back().elems,
                          A, h->arena, flags, st);
    }
    if (e == hipSuccess && !p.pack.empty())
        e = launch_pack(dp.d_pack, (int)p.pack.size(), p.pack.back().elem_begin + p.pack.back().elems,
                        A, h->arena, flags, st);
    mark(2);
    if (e == hipSuccess)
        e = launch_leaves(mode, p.tile_cfg, dp.d_leaves, (int)p.leaves.size(), p.total_tiles, A, C_packed, h->arena,
                          flags, h->chunk, st);
    if (e == hipSuccess && !p.fb_leaves.empty())
        e = launch_fallback_leaves(dp.d_fb_leaves, (int)p.fb_leaves.size(), p.fb_tiles, A, C_packed,
                                   h->arena, flags, h->chunk, st);
    mark(3);
    for (size_t l = 0; e == hipSuccess && l < p.combine.size(); ++l) {
        const auto& lv = p.combine[l];
        e = launch_combine(mode, dp.d_combine[l], (int)lv.size(), lv.back().elem_begin + lv.back().elems,
                           C_packed, h->arena, flags, st);
    }
    mark(4);
    if (e == hipSuccess && h->residual)
        e = launch_residual(mode, A, m, n, lda, C_packed, h->seed, res_work, res, st);
    mark(5);
    if (e != hipSuccess) return ATA_ERR_HIP;

    fill_report(h->report, p);
    h->last_stream = st;
    h->pending_flags = p.fallback;
    h->pending_residual = h->residual;
    h->last_flags = flags;
    h->last_residual = res;
    h->last_nodes = (int64_t)p.nodes.size();
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
    ata_status_t s = ensure(buf, cap, bytes);
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

ata_status_t ata_gram_batched(ata_handle_t h, int64_t batch, const void* const* A,
                              const int64_t* m, const int64_t* n, const int64_t* lda,
                              ata_dtype_t dtype, void* const* C_packed, void* stream) {
    (void)stream;
    if (!h || batch <= 0 || !A || !m || !n || !lda || !C_packed || !valid_dtype(dtype))
        return ATA_ERR_INVALID_VALUE;
    return ATA_ERR_NOT_SUPPORTED;
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
