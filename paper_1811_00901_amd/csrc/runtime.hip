// Host runtime of the spin-image library: the C ABI of include/si.h.
//
// Scene construction, parameter validation, schedule (chunk-table) caching,
// the generation launch and its statistics.  The paper's master process
// (Section 3, the master's algorithm) becomes host code that computes a chunk
// table once per schedule, plus a device-global counter that the persistent
// workgroups of the spin kernel advance to claim chunks.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "scene_build.h"
#include "adaptive.h"

namespace si {

// ---------------------------------------------------------------- errors --
static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

si_status fail(si_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

si_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? SI_E_OOM : SI_E_DEVICE;
}

// Entry points that upload host data or wait on the host cannot be captured
// into a graph: a replay would repeat an upload from host storage that later
// calls refill, and the waits are not allowed under capture.  They refuse a
// capturing stream before enqueuing anything.
si_status refuse_capture(hipStream_t s, const char* what) {
    hipStreamCaptureStatus c = hipStreamCaptureStatusNone;
    const hipError_t e = hipStreamIsCapturing(s, &c);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (c != hipStreamCaptureStatusNone)
        return fail(SI_E_UNSUPPORTED,
                    std::string(what) + " cannot be captured into a graph: it uploads host data "
                    "or waits on the host (si_generate_batched with use_graph = 1 replays "
                    "a graph of its own)");
    return SI_OK;
}

hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s) {
    if (const char* lim = getenv("SI_TEST_ALLOC_FAIL")) {
        if (bytes >= (size_t)strtoull(lim, nullptr, 10)) {
            *p = nullptr;
            return hipErrorOutOfMemory;
        }
    }
    return hipMallocAsync(p, bytes, s);
}

// caller-supplied events recorded around spin-kernel launches (this thread)
static thread_local hipEvent_t g_ev_begin = nullptr;
static thread_local hipEvent_t g_ev_end = nullptr;

void user_kernel_events(hipEvent_t* begin, hipEvent_t* end) {
    *begin = g_ev_begin;
    *end = g_ev_end;
}

static thread_local int32_t g_emu_every = 0;
static thread_local float g_emu_slowdown = 1.0f;
static thread_local int32_t g_emu_busy = 0;
static thread_local int32_t g_emu_place = SI_EMU_EVERY;
static thread_local std::vector<float> g_weights;

void apply_emulated_workers(LaunchDesc& d) {
    d.emu_every = g_emu_every;
    d.emu_extra = g_emu_slowdown - 1.0f;
    d.emu_busy = g_emu_busy;
    d.emu_place = g_emu_place;
}

const std::vector<float>& worker_weights() { return g_weights; }

// --------------------------------------------------------- device state --
}  // namespace si

namespace {

constexpr int kCounterSlots = 64;
constexpr int kCounterStride = 32;  // u32 words between slots (128 bytes)

}  // namespace

// Work-counter slots of the generation launches, one copy per device (zero
// when the code object is loaded; each launch leaves its slot at zero).
static __device__ __align__(256) uint32_t work_counters[kCounterSlots * kCounterStride];

namespace si {

static std::mutex g_mu;
static std::map<int, DeviceState> g_dev;

// Set-up of a device: attributes and the address of its counter slots; no
// allocation, no synchronisation and no stream work.
si_status device_state(DeviceState** out) {
    int dev = 0;
    SI_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceState& st = g_dev[dev];
    if (!st.ready) {
        SI_HIP(hipDeviceGetAttribute(&st.n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess &&
            khz > 0)
            st.wall_khz = khz;
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                hipSuccess && lds > 0)
            st.max_lds = std::min(lds, 65536);
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t keep = UINT64_MAX;  // stream-ordered temporaries stay cached
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
        void* slots = nullptr;
        SI_HIP(hipGetSymbolAddress(&slots, HIP_SYMBOL(work_counters)));
        st.counters = static_cast<uint32_t*>(slots);
        st.ready = true;
    }
    *out = &st;
    return SI_OK;
}

uint32_t* take_counter(DeviceState* st) {
    std::lock_guard<std::mutex> lk(g_mu);
    const uint32_t k = st->next_slot++ % kCounterSlots;
    return st->counters + (size_t)k * kCounterStride;
}

static bool finite_f(float v) { return isfinite(v); }

// ------------------------------------------------------------ parameters --
si_status make_params(const si_params* prm, SpinParams* out, double* radius) {
    if (!prm) return fail(SI_E_INVALID, "params is NULL");
    if (prm->W < 2 || prm->W > 64) return fail(SI_E_INVALID, "W must be in [2, 64]");
    if (!finite_f(prm->bin) || !(prm->bin > 0.0f))
        return fail(SI_E_INVALID, "bin must be finite and > 0");
    if (!finite_f(prm->support_angle) || !(prm->support_angle >= 0.0f))
        return fail(SI_E_INVALID, "support_angle must be finite and >= 0");
    if (prm->mode != SI_BIN_BILINEAR && prm->mode != SI_BIN_CEIL)
        return fail(SI_E_INVALID, "mode must be SI_BIN_BILINEAR or SI_BIN_CEIL");
    const double B = prm->bin;
    const double half = 0.5 * prm->W;
    const double hi = prm->mode == SI_BIN_CEIL ? B * (half + 1.0) : B * half;
    const double lo = B * (1.0 - half);
    const double amax = B * (prm->W - 1.0);
    SpinParams p;
    p.W = prm->W;
    p.mode = prm->mode;
    p.half = (float)half;
    p.inv_bin = (float)(1.0 / B);
    p.beta_lo = (float)lo;
    p.beta_hi = (float)hi;
    p.alpha2_max = (float)(amax * amax);
    const double S = prm->support_angle;
    p.angle_on = S < M_PI ? 1 : 0;
    p.cos_s = (float)cos(S);
    const double R = sqrt(std::max(fabs(hi), fabs(lo)) * std::max(fabs(hi), fabs(lo)) + amax * amax);
    *radius = R;
    // culling radius: any pair the float32 test can accept lies within it
    p.radius = (float)(R * (1.0 + 1e-5));
    p.reach = 0;
    *out = p;
    return SI_OK;
}

// ----------------------------------------------------------- chunk tables --
int64_t chunk_sizes(int kind, int64_t N, int P, int min_chunk, float divisor, int64_t* starts,
                    int64_t cap) {
    // Returns the number of chunks; writes starts[0..n] when cap allows (n+1 entries).
    int64_t n = 0, pos = 0;
    auto put = [&](int64_t c) {
        if (starts && n < cap) starts[n] = pos;
        pos += c;
        ++n;
    };
    const int64_t mc = std::max(1, min_chunk);
    if (kind == SI_SCHED_STATIC) {
        const int64_t q = N / P, r = N % P;
        for (int k = 0; k < P; ++k) put(q + (k < r ? 1 : 0));
    } else if (kind == SI_SCHED_SS) {
        for (int64_t R = N; R > 0;) {
            const int64_t c = std::min(mc, R);
            put(c);
            R -= c;
        }
    } else if (kind == SI_SCHED_GSS) {
        for (int64_t R = N; R > 0;) {
            const int64_t c = std::min(std::max((R + P - 1) / P, mc), R);
            put(c);
            R -= c;
        }
    } else if (kind == SI_SCHED_TSS) {
        // trapezoid self-scheduling: sizes fall linearly from F = ceil(N / 2P)
        // towards L over C = ceil(2N / (F + L)) chunks, chunk i of
        // ceil(F - i delta) with the real step delta = (F - L) / (C - 1)
        const int64_t L = mc;
        const int64_t F = std::max((N + 2 * (int64_t)P - 1) / (2 * (int64_t)P), L);
        const int64_t C = (2 * N + F + L - 1) / (F + L);
        const double delta = C > 1 ? (double)(F - L) / (double)(C - 1) : 0.0;
        int64_t i = 0;
        for (int64_t R = N; R > 0; ++i) {
            const int64_t c = std::max((int64_t)ceil((double)F - (double)i * delta), L);
            const int64_t k = std::min(c, R);
            put(k);
            R -= k;
        }
    } else if (kind == SI_SCHED_FAC_PROB) {
        // probabilistic factoring: batch j of P chunks of ceil(R_j / (x_j P)),
        // x_j from b_j = P cv / (2 sqrt(R_j)), cv = sigma / mu of the
        // iteration cost (the first batch's ratio differs from the later ones')
        const double cv = (double)divisor;
        bool first = true;
        for (int64_t R = N; R > 0;) {
            const double b = (double)P * cv / (2.0 * sqrt((double)R));
            const double x = first ? 1.0 + b * b + b * sqrt(b * b + 2.0)
                                   : 2.0 + b * b + b * sqrt(b * b + 4.0);
            first = false;
            const int64_t c = std::max((int64_t)ceil((double)R / (x * (double)P)), mc);
            for (int k = 0; k < P && R > 0; ++k) {
                const int64_t cc = std::min(c, R);
                put(cc);
                R -= cc;
            }
        }
    } else {  // FAC / LEARNED tables over equal-cost units
        const double x = divisor > 0.0f ? (double)divisor : 2.0;
        for (int64_t R = N; R > 0;) {
            const int64_t c = std::max((int64_t)ceil((double)R / (x * (double)P)), mc);
            for (int k = 0; k < P && R > 0; ++k) {
                const int64_t cc = std::min(c, R);
                put(cc);
                R -= cc;
            }
        }
    }
    if (starts && n < cap) starts[n] = pos;
    return n;
}

si_status get_table(DeviceState* st, int kind, int64_t N, int P, int min_chunk,
                           float divisor, Chunk** out, int* n_out, hipStream_t s, void** entry) {
    // the parameter: FAC's divisor (0 = 2), FAC_PROB's cost variation (0 kept)
    uint32_t dbits;
    const float dv = kind == SI_SCHED_FAC_PROB ? divisor : divisor > 0.0f ? divisor : 2.0f;
    memcpy(&dbits, &dv, 4);
    const int kk = kind;
    const bool param = kk == SI_SCHED_FAC || kk == SI_SCHED_FAC_PROB;
    auto key = std::make_tuple(kk, N, P, kind == SI_SCHED_STATIC ? 0 : std::max(1, min_chunk),
                               param ? dbits : 0u);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = st->tables.find(key);
    if (it != st->tables.end()) {
        DeviceState::Table& t = it->second;
        t.tick = ++st->table_tick;
        SI_HIP(hipStreamWaitEvent(s, t.ready, 0));  // uploaded on another stream
        ++t.pins;
        *out = t.dev;
        *n_out = t.n;
        *entry = &t;
        return SI_OK;
    }
    const int64_t n = chunk_sizes(kind, N, P, min_chunk, dv, nullptr, 0);
    if (n > INT32_MAX) return fail(SI_E_INVALID, "schedule has too many chunks");
    std::vector<int64_t> starts(n + 1);
    chunk_sizes(kind, N, P, min_chunk, dv, starts.data(), n + 1);
    // evict the least recently used table not held by a call in progress,
    // once the work that reads it is done
    auto lru = st->tables.end();
    if (st->tables.size() >= 64)
        for (auto i = st->tables.begin(); i != st->tables.end(); ++i)
            if (i->second.pins == 0 && (lru == st->tables.end() || i->second.tick < lru->second.tick))
                lru = i;
    if (lru != st->tables.end()) {
        DeviceState::Table& t = lru->second;
        for (auto& u : t.uses) {
            SI_HIP(hipEventSynchronize(u.second));
            (void)hipEventDestroy(u.second);
        }
        SI_HIP(hipEventSynchronize(t.ready));
        (void)hipEventDestroy(t.ready);
        SI_HIP(hipFreeAsync(t.dev, s));
        st->tables.erase(lru);
    }
    // the host table into the pinned staging buffer (after its previous copy)
    const size_t bytes = sizeof(Chunk) * (size_t)std::max<int64_t>(n, 1);
    if (!st->stage_done) SI_HIP(hipEventCreateWithFlags(&st->stage_done, hipEventDisableTiming));
    SI_HIP(hipEventSynchronize(st->stage_done));
    if (st->stage_bytes < bytes) {
        if (st->stage) SI_HIP(hipHostFree(st->stage));
        st->stage = nullptr;
        st->stage_bytes = 0;
        const size_t cap = std::max(bytes, (size_t)1 << 20);
        SI_HIP(hipHostMalloc(&st->stage, cap, hipHostMallocDefault));
        st->stage_bytes = cap;
    }
    Chunk* h = static_cast<Chunk*>(st->stage);
    for (int64_t i = 0; i < n; ++i) {
        h[i].item = 0;
        h[i].start = (int32_t)starts[i];
        h[i].end = (int32_t)starts[i + 1];
    }
    DeviceState::Table t;
    t.n = (int)n;
    t.tick = ++st->table_tick;
    SI_HIP(pool_alloc((void**)&t.dev, bytes, s));
    hipError_t e = n ? hipMemcpyAsync(t.dev, h, sizeof(Chunk) * n, hipMemcpyHostToDevice, s)
                     : hipSuccess;
    if (e == hipSuccess) e = hipEventRecord(st->stage_done, s);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&t.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(t.ready, s);
    if (e != hipSuccess) {
        (void)hipFreeAsync(t.dev, s);
        if (t.ready) (void)hipEventDestroy(t.ready);
        return hip_fail(e, "chunk table upload");
    }
    t.pins = 1;
    DeviceState::Table& in = st->tables[key] = t;
    *out = in.dev;
    *n_out = in.n;
    *entry = &in;
    return SI_OK;
}

si_status table_used(DeviceState* st, void* entry, hipStream_t s, bool launched) {
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceState::Table* t = static_cast<DeviceState::Table*>(entry);
    --t->pins;
    if (!launched) return SI_OK;
    hipEvent_t& ev = t->uses[s];
    if (!ev) SI_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    SI_HIP(hipEventRecord(ev, s));
    return SI_OK;
}

// ------------------------------------------------------------------ scene --
SceneView view_of(const Scene& s) {
    SceneView v;
    v.pos = s.pos;
    v.nrm = s.nrm;
    v.sub_start = s.sub_start;
    v.inv = s.inv;
    for (int a = 0; a < 3; ++a) {
        v.dims[a] = s.dims[a];
        v.origin[a] = s.origin[a];
    }
    v.h = s.h;
    v.M = (int32_t)s.M;
    return v;
}

// The scenes of one si_build_scenes call share one allocation of their
// arrays (mem is its base for all of them); it is released with the last of
// them.  Counts of the scenes still holding each shared allocation:
static std::mutex g_shared_mu;
static std::map<void*, int64_t> g_shared_refs;

// The scene's arrays come from the device's stream-ordered pool (which keeps
// freed memory cached), so building a scene per frame costs no allocation
// round trips.  Frees are ordered on `stream`.
static void free_scene_mem(Scene* sc, hipStream_t stream) {
    if (!sc) return;
    if (sc->mem) {
        bool last = true;
        {
            std::lock_guard<std::mutex> lk(g_shared_mu);
            auto it = g_shared_refs.find(sc->mem);
            if (it != g_shared_refs.end()) {
                last = --it->second == 0;
                if (last) g_shared_refs.erase(it);
            }
        }
        if (last) (void)hipFreeAsync(sc->mem, stream);
    }
    sc->mem = nullptr;
    sc->pos = sc->nrm = nullptr;
    sc->sub_start = sc->inv = nullptr;
}

static size_t rup256(size_t b) { return (b + 255) & ~(size_t)255; }

// A scene's grid from the bounding box of its finite coordinates (hb: lo
// xyz, hi xyz) and the largest support radius it will serve: cells of edge
// R (1 + 2e-5) / kSub, enlarged while the grid would exceed kMaxCells; a
// radius <= 0 (or no finite point) gives one cell, the brute-force loop.
static void scene_grid(Scene* sc, const float hb[6], float max_support_radius) {
    double lo[3], ext[3];
    bool any = true;
    for (int a = 0; a < 3; ++a) {
        if (!(hb[a] <= hb[3 + a])) any = false;
        lo[a] = any ? (double)hb[a] : 0.0;
    }
    for (int a = 0; a < 3; ++a) ext[a] = any ? (double)hb[3 + a] - lo[a] : 0.0;
    for (int a = 0; a < 3; ++a) sc->origin[a] = any ? hb[a] : 0.0f;

    if (max_support_radius > 0.0f && any) {
        // margin 2e-5 > the 1e-5 of the culling radius: reach stays <= kSub
        double h = (double)max_support_radius * (1.0 + 2e-5) / kSub;
        for (;;) {
            int64_t cells = 1;
            for (int a = 0; a < 3; ++a) {
                const int64_t d = (int64_t)floor(ext[a] / h) + 1;
                sc->dims[a] = (int32_t)d;
                cells *= d;
            }
            if (cells <= kMaxCells) {
                sc->n_cells = cells;
                break;
            }
            h *= std::cbrt((double)cells / (double)kMaxCells) * 1.01;
        }
        sc->h = h;
        sc->max_radius = max_support_radius;
    } else {
        sc->h = std::max({ext[0], ext[1], ext[2], 0.0}) + 1.0;
        sc->dims[0] = sc->dims[1] = sc->dims[2] = 1;
        sc->n_cells = 1;
        sc->max_radius = 0.0f;
    }
}

// Bytes of the scene's four arrays (each 256-byte aligned).
static size_t scene_bytes(const Scene* sc) {
    const int64_t M = sc->M, n_keys = sc->n_cells * kSubX;
    return 2 * rup256(sizeof(float4) * M) + rup256(sizeof(int32_t) * M) +
           rup256(sizeof(int32_t) * (n_keys + 1));
}

// Point the scene's arrays into m (scene_bytes(sc) bytes).
static void scene_place(Scene* sc, char* m) {
    const size_t b_pos = rup256(sizeof(float4) * sc->M), b_inv = rup256(sizeof(int32_t) * sc->M);
    sc->pos = reinterpret_cast<float4*>(m);
    sc->nrm = reinterpret_cast<float4*>(m + b_pos);
    sc->inv = reinterpret_cast<int32_t*>(m + 2 * b_pos);
    sc->sub_start = reinterpret_cast<int32_t*>(m + 2 * b_pos + b_inv);
}

// The scene's four arrays, in one allocation from the device's pool.
static hipError_t scene_alloc(Scene* sc, hipStream_t s) {
    hipError_t e = pool_alloc(&sc->mem, scene_bytes(sc), s);
    if (e != hipSuccess) {
        sc->mem = nullptr;
        return e;
    }
    scene_place(sc, static_cast<char*>(sc->mem));
    return hipSuccess;
}

}  // namespace si

using namespace si;

extern "C" {

si_status si_build_scene(const float* points_xyz, const float* normals_xyz, int64_t M,
                         float max_support_radius, void* hip_stream, si_scene** out) {
    if (!out) return fail(SI_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!points_xyz || !normals_xyz) return fail(SI_E_INVALID, "points or normals is NULL");
    if (M <= 0 || M >= INT32_MAX) return fail(SI_E_INVALID, "M must be in [1, 2^31 - 1)");
    if (!isfinite(max_support_radius)) return fail(SI_E_INVALID, "max_support_radius not finite");
    hipStream_t s = (hipStream_t)hip_stream;
    si_status rc = refuse_capture(s, "si_build_scene");
    if (rc != SI_OK) return rc;
    DeviceState* st;
    rc = device_state(&st);
    if (rc != SI_OK) return rc;

    si_scene* sc = new (std::nothrow) si_scene();
    if (!sc) return fail(SI_E_OOM, "host allocation failed");
    sc->M = M;
    SI_HIP(hipGetDevice(&sc->device));

    // ---- bounding box (the one synchronisation) ----
    float* bb = nullptr;
    hipError_t e = pool_alloc((void**)&bb, sizeof(float) * (8 + 6 * 1024), s);
    if (e != hipSuccess) { delete sc; return hip_fail(e, "bounding-box scratch"); }
    float hb[6];
    e = launch_bbox(points_xyz, M, bb, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hb, bb, sizeof(hb), hipMemcpyDeviceToHost, s);
    (void)hipFreeAsync(bb, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { delete sc; return hip_fail(e, "scene bounding box"); }

    scene_grid(sc, hb, max_support_radius);

    // ---- bin, scan, scatter ----
    int32_t *key_of = nullptr, *rank = nullptr, *counts = nullptr, *tmp = nullptr;
    const int64_t n_keys = sc->n_cells * kSubX;
    const int64_t ntmp = scan_tmp_elems(n_keys);
    // two pool allocations: the scene's arrays, and temporaries that return
    // to the pool once the stream has used them
    const size_t b_inv = rup256(sizeof(int32_t) * M);
    const size_t b_key = rup256(sizeof(int32_t) * n_keys);
    char* tmem = nullptr;
    e = scene_alloc(sc, s);
    if (e == hipSuccess)
        e = pool_alloc((void**)&tmem, 2 * b_inv + b_key + rup256(sizeof(int32_t) * ntmp), s);
    if (e == hipSuccess) {
        key_of = reinterpret_cast<int32_t*>(tmem);
        rank = reinterpret_cast<int32_t*>(tmem + b_inv);
        counts = reinterpret_cast<int32_t*>(tmem + 2 * b_inv);
        tmp = reinterpret_cast<int32_t*>(tmem + 2 * b_inv + b_key);
    }
    auto cleanup = [&]() {
        if (tmem) (void)hipFreeAsync(tmem, s);
    };
    if (e == hipSuccess) e = launch_fill(counts, n_keys, 0, s);
    if (e == hipSuccess) e = launch_bin_points(points_xyz, M, *sc, key_of, rank, counts, s);
    if (e == hipSuccess) e = launch_scan(counts, sc->sub_start, n_keys, tmp, ntmp, s);
    if (e == hipSuccess)
        e = launch_scatter(points_xyz, normals_xyz, M, key_of, rank, sc->sub_start, *sc, s);
    if (e == hipSuccess) e = hipGetLastError();
    cleanup();
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        free_scene_mem(sc, s);
        delete sc;
        return hip_fail(e, "scene build");
    }
    *out = sc;
    return SI_OK;
}

// Bounding-box blocks per scene and sub-batch bounds of a batched build.
static constexpr int64_t kBBoxBlocksPerScene = 64;
static constexpr int64_t kBuildKeys = int64_t(1) << 27;
static constexpr int64_t kBuildPoints = int64_t(1) << 28;

si_status si_build_scenes(const si_scene_desc* descs, int32_t n, void* hip_stream,
                          si_scene** out) {
    if (n < 0) return fail(SI_E_INVALID, "n must be >= 0");
    if (n == 0) return SI_OK;
    if (!descs || !out) return fail(SI_E_INVALID, "descs or out is NULL");
    for (int i = 0; i < n; ++i) out[i] = nullptr;
    for (int i = 0; i < n; ++i) {
        const si_scene_desc& d = descs[i];
        const std::string at = "scene " + std::to_string(i) + ": ";
        if (!d.points_xyz || !d.normals_xyz)
            return fail(SI_E_INVALID, at + "points or normals is NULL");
        if (d.M <= 0 || d.M >= INT32_MAX)
            return fail(SI_E_INVALID, at + "M must be in [1, 2^31 - 1)");
        if (!isfinite(d.max_support_radius))
            return fail(SI_E_INVALID, at + "max_support_radius not finite");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    si_status rc = refuse_capture(s, "si_build_scenes");
    if (rc != SI_OK) return rc;
    DeviceState* st;
    rc = device_state(&st);
    if (rc != SI_OK) return rc;
    int dev = 0;
    SI_HIP(hipGetDevice(&dev));

    std::vector<si_scene*> scenes(n, nullptr);
    auto discard = [&]() {
        (void)hipStreamSynchronize(s);
        for (si_scene*& sc : scenes) {
            if (sc) free_scene_mem(sc, s);
            delete sc;
            sc = nullptr;
        }
    };
    for (int i = 0; i < n; ++i) {
        scenes[i] = new (std::nothrow) si_scene();
        if (!scenes[i]) {
            discard();
            return fail(SI_E_OOM, "host allocation failed");
        }
        scenes[i]->M = descs[i].M;
        scenes[i]->device = dev;
    }

    // ---- bounding boxes of all scenes (one synchronisation) ----
    std::vector<BuildItem> items(n);
    std::vector<int64_t> blk_off(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        memset(&items[i], 0, sizeof(BuildItem));
        items[i].xyz = descs[i].points_xyz;
        items[i].nrm = descs[i].normals_xyz;
        items[i].M = descs[i].M;
        blk_off[i + 1] = blk_off[i] + std::min(kBBoxBlocksPerScene, (descs[i].M + 255) / 256);
    }
    const int64_t n_blk = blk_off[n];
    std::vector<float> hb(6 * (size_t)n);
    {
        const size_t b_it = rup256(sizeof(BuildItem) * n);
        const size_t b_off = rup256(sizeof(int64_t) * (n + 1));
        const size_t b_part = rup256(sizeof(float) * 6 * n_blk);
        char* m = nullptr;
        hipError_t e = pool_alloc((void**)&m, b_it + b_off + b_part + sizeof(float) * 6 * n, s);
        if (e == hipSuccess) {
            BuildItem* d_it = reinterpret_cast<BuildItem*>(m);
            int64_t* d_off = reinterpret_cast<int64_t*>(m + b_it);
            float* d_part = reinterpret_cast<float*>(m + b_it + b_off);
            float* d_box = reinterpret_cast<float*>(m + b_it + b_off + b_part);
            e = hipMemcpyAsync(d_it, items.data(), sizeof(BuildItem) * n, hipMemcpyHostToDevice,
                               s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_off, blk_off.data(), sizeof(int64_t) * (n + 1),
                                   hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = launch_bbox_multi(d_it, d_off, n, n_blk, d_part, d_box, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(hb.data(), d_box, sizeof(float) * 6 * n,
                                   hipMemcpyDeviceToHost, s);
            (void)hipFreeAsync(m, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
        if (e != hipSuccess) {
            discard();
            return hip_fail(e, "batched bounding boxes");
        }
    }

    // ---- grids and the scenes' arrays (one shared allocation) ----
    size_t total_bytes = 0;
    for (int i = 0; i < n; ++i) {
        scene_grid(scenes[i], &hb[6 * (size_t)i], descs[i].max_support_radius);
        total_bytes += scene_bytes(scenes[i]);
    }
    void* shared = nullptr;
    {
        const hipError_t e = pool_alloc(&shared, total_bytes, s);
        if (e != hipSuccess) {
            discard();
            return hip_fail(e, "scene arrays");
        }
        std::lock_guard<std::mutex> lk(g_shared_mu);
        g_shared_refs[shared] = n;
    }
    size_t at = 0;
    for (int i = 0; i < n; ++i) {
        si_scene* sc = scenes[i];
        sc->mem = shared;
        scene_place(sc, static_cast<char*>(shared) + at);
        at += scene_bytes(sc);
        items[i].g = grid_of(*sc);
        items[i].pos = sc->pos;
        items[i].nr = sc->nrm;
        items[i].inv = sc->inv;
        items[i].sub_start = sc->sub_start;
    }

    // ---- bin, scan and scatter in bounded sub-batches ----
    // SI_TEST_BUILD_KEYS, a key count, lowers the key bound of a sub-batch: a
    // test hook for builds that take several sub-batches
    int64_t key_cap = kBuildKeys;
    if (const char* v = getenv("SI_TEST_BUILD_KEYS")) {
        const long long k = strtoll(v, nullptr, 10);
        if (k > 0) key_cap = k;
    }
    for (int b0 = 0; b0 < n;) {
        int64_t n_keys = 0, n_pts = 0;
        int b1 = b0;
        while (b1 < n) {
            const int64_t k = scenes[b1]->n_cells * kSubX;
            if (b1 > b0 && (n_keys + k > key_cap || n_pts + descs[b1].M > kBuildPoints)) break;
            items[b1].key_base = n_keys;
            n_keys += k;
            n_pts += descs[b1].M;
            ++b1;
        }
        const int nb = b1 - b0;
        std::vector<int64_t> pt_off(nb + 1, 0), sub_off(nb + 1, 0);
        for (int j = 0; j < nb; ++j) {
            pt_off[j + 1] = pt_off[j] + descs[b0 + j].M;
            sub_off[j + 1] = sub_off[j] + scenes[b0 + j]->n_cells * kSubX + 1;
        }
        const int64_t ntmp = scan_tmp_elems(n_keys);
        const size_t b_it = rup256(sizeof(BuildItem) * nb);
        const size_t b_off = rup256(sizeof(int64_t) * (nb + 1));
        const size_t b_pt = rup256(sizeof(int32_t) * n_pts);
        const size_t b_cnt = rup256(sizeof(int32_t) * n_keys);
        const size_t b_scan = rup256(sizeof(int32_t) * (n_keys + 1));
        char* m = nullptr;
        hipError_t e = pool_alloc((void**)&m,
                                  b_it + 2 * b_off + 2 * b_pt + b_cnt + b_scan +
                                      sizeof(int32_t) * ntmp, s);
        if (e == hipSuccess) {
            BuildItem* d_it = reinterpret_cast<BuildItem*>(m);
            int64_t* d_pt = reinterpret_cast<int64_t*>(m + b_it);
            int64_t* d_sub = reinterpret_cast<int64_t*>(m + b_it + b_off);
            char* t = m + b_it + 2 * b_off;
            int32_t* key_of = reinterpret_cast<int32_t*>(t);
            int32_t* rank = reinterpret_cast<int32_t*>(t + b_pt);
            int32_t* counts = reinterpret_cast<int32_t*>(t + 2 * b_pt);
            int32_t* gscan = reinterpret_cast<int32_t*>(t + 2 * b_pt + b_cnt);
            int32_t* tmp = reinterpret_cast<int32_t*>(t + 2 * b_pt + b_cnt + b_scan);
            e = hipMemcpyAsync(d_it, items.data() + b0, sizeof(BuildItem) * nb,
                               hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_pt, pt_off.data(), sizeof(int64_t) * (nb + 1),
                                   hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_sub, sub_off.data(), sizeof(int64_t) * (nb + 1),
                                   hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = launch_build_multi(d_it, d_pt, d_sub, nb, n_pts, n_keys, key_of, rank,
                                       counts, gscan, tmp, s);
            (void)hipFreeAsync(m, s);
            // the host tables are staged from pageable memory: wait before they go
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
        if (e != hipSuccess) {
            discard();
            return hip_fail(e, "batched scene build");
        }
        b0 = b1;
    }
    for (int i = 0; i < n; ++i) out[i] = scenes[i];
    return SI_OK;
}

void si_free_scene(si_scene* scene) {
    if (!scene) return;
    // work using the scene has completed (caller's contract); the device-wide
    // synchronisation also covers the build's own kernels, which may still be
    // queued on a stream that does not synchronise with the null stream
    (void)hipDeviceSynchronize();
    drop_graphs_of(scene->serial);  // graphs hold its grid and arrays by value
    free_scene_mem(scene, nullptr);
    delete scene;
}

si_status si_scene_info_get(const si_scene* scene, si_scene_info* out) {
    if (!scene || !out) return fail(SI_E_INVALID, "NULL argument");
    out->M = scene->M;
    out->cell_size = (float)scene->h;
    out->max_support_radius = scene->max_radius;
    for (int a = 0; a < 3; ++a) {
        out->dims[a] = scene->dims[a];
        out->origin[a] = scene->origin[a];
    }
    out->n_cells = scene->n_cells;
    return SI_OK;
}

si_status si_support_radius(const si_params* params, float* radius) {
    if (!radius) return fail(SI_E_INVALID, "radius is NULL");
    SpinParams p;
    double R;
    si_status rc = make_params(params, &p, &R);
    if (rc != SI_OK) return rc;
    float r = (float)R;
    if ((double)r < R) r = nextafterf(r, INFINITY);  // never below the true radius
    *radius = r;
    return SI_OK;
}

si_status si_chunk_table(int32_t kind, int64_t N, int32_t P, int32_t min_chunk,
                         float fac_divisor, int64_t* starts_out, int64_t cap,
                         int64_t* n_chunks) {
    if (kind < SI_SCHED_STATIC || kind > SI_SCHED_FAC_PROB || kind == SI_SCHED_LEARNED)
        return fail(SI_E_INVALID, "bad kind");
    if (N < 0 || P < 1) return fail(SI_E_INVALID, "N must be >= 0 and P >= 1");
    if (fac_divisor < 0.0f || !isfinite(fac_divisor)) return fail(SI_E_INVALID, "bad divisor");
    const int64_t n = chunk_sizes(kind, N, P, min_chunk, fac_divisor, nullptr, 0);
    if (n_chunks) *n_chunks = n;
    if (starts_out) {
        if (cap < n + 1) return fail(SI_E_INVALID, "starts_out capacity too small");
        chunk_sizes(kind, N, P, min_chunk, fac_divisor, starts_out, cap);
    }
    return SI_OK;
}

}  // extern "C"

// --------------------------------------------------------------- generate --
namespace si {

// Images per candidate pass: 4 keeps the per-image values of a group in
// scalar registers; W = 64 images are 16 KB each, so two per pass.
int default_group(int W) { return W >= 64 ? 2 : 4; }

int32_t spread_mult(int64_t full) {
    if (full <= 1 || full >= INT32_MAX) return 0;
    int64_t m = (int64_t)llround(0.6180339887498949 * (double)full) | 1;
    auto gcd = [](int64_t a, int64_t b) {
        while (b) { const int64_t t = a % b; a = b; b = t; }
        return a;
    };
    while (gcd(m, full) != 1) m += 2;
    return (int32_t)(m % full);
}

// Largest group <= the requested one whose accumulators fit the LDS limit.
int fit_group(DeviceState* st, int group, int max_w2) {
    const size_t static_lds = 20480;  // kernel's own shared arrays (~14 KB), rounded up
    while (group > 1 && spin_lds_bytes(max_w2, group) + static_lds > (size_t)st->max_lds) --group;
    return group;
}

si_status run_launch(DeviceState* st, LaunchDesc& d, int n_wg, int max_w2, si_stats* stats,
                     hipStream_t s, int sched_used) {
    d.max_w2 = max_w2;
    d.counter = take_counter(st);
    d.ovf_limit = 65536u;
    if (const char* lim = getenv("SI_TEST_OVERFLOW_LIMIT")) d.ovf_limit = (uint32_t)atol(lim);
    unsigned long long* dev_stats = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (stats) {
        const size_t words = 5 + (size_t)n_wg;
        SI_HIP(hipMalloc(&dev_stats, sizeof(unsigned long long) * words));
        SI_HIP(launch_fill(reinterpret_cast<int32_t*>(dev_stats), (int64_t)(2 * words), 0, s));
        d.stat_tested = dev_stats;
        d.stat_support = dev_stats + 1;
        d.stat_invalid = reinterpret_cast<uint32_t*>(dev_stats + 2);
        d.stat_overflow = reinterpret_cast<uint32_t*>(dev_stats + 3);
        d.stat_chunks = reinterpret_cast<uint32_t*>(dev_stats + 4);
        d.wg_ns = dev_stats + 5;
        SI_HIP(hipEventCreate(&ev0));
        SI_HIP(hipEventCreate(&ev1));
        SI_HIP(hipEventRecord(ev0, s));
    } else {
        d.stat_tested = d.stat_support = nullptr;
        d.stat_invalid = d.stat_overflow = nullptr;
        d.stat_chunks = nullptr;
        d.wg_ns = nullptr;
    }
    if (g_ev_begin) SI_HIP(hipEventRecord(g_ev_begin, s));
    hipError_t e = launch_spin(d, n_wg, s);
    if (e == hipSuccess && g_ev_end) e = hipEventRecord(g_ev_end, s);
    if (e != hipSuccess) {
        (void)hipFree(dev_stats);
        return hip_fail(e, "spin-image launch");
    }
    if (!stats) return SI_OK;
    SI_HIP(hipEventRecord(ev1, s));
    std::vector<unsigned long long> h(5 + (size_t)n_wg);
    SI_HIP(hipMemcpyAsync(h.data(), dev_stats, sizeof(unsigned long long) * h.size(),
                          hipMemcpyDeviceToHost, s));
    SI_HIP(hipStreamSynchronize(s));
    float ms = 0.0f;
    SI_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    (void)hipFree(dev_stats);
    stats->kernel_ms = ms;
    stats->pairs_tested = h[0];
    stats->pairs_in_support = h[1];
    stats->n_invalid = (int32_t)(uint32_t)h[2];
    stats->n_overflow = (int32_t)(uint32_t)h[3];
    stats->sched_used = sched_used;
    stats->n_wg = n_wg;
    stats->n_chunks = d.n_chunks;
    if (d.n_chunks_dev) {
        int32_t nc = 0;
        SI_HIP(hipMemcpy(&nc, d.n_chunks_dev, sizeof(nc), hipMemcpyDeviceToHost));
        stats->n_chunks = nc;
    }
    if (d.rule) stats->n_chunks = (int32_t)(uint32_t)h[4];
    if (stats->wg_busy_ns) {
        const int n = std::min(stats->wg_busy_cap, n_wg);
        for (int i = 0; i < n; ++i)
            stats->wg_busy_ns[i] = (uint64_t)((double)h[5 + i] * 1e6 / (double)st->wall_khz);
    }
    if (stats->n_invalid) return fail(SI_E_INVALID, "oriented_idx holds indices outside [0, M)");
    return SI_OK;
}

si_status check_sched(const si_sched* sc) {
    if (!sc) return fail(SI_E_INVALID, "sched is NULL");
    if (sc->kind < SI_SCHED_STATIC || sc->kind > SI_SCHED_AF)
        return fail(SI_E_INVALID, "unknown schedule kind");
    if (sc->num_workgroups < 0) return fail(SI_E_INVALID, "num_workgroups must be >= 0");
    if (sc->min_chunk < 0) return fail(SI_E_INVALID, "min_chunk must be >= 0");
    if (!isfinite(sc->fac_divisor) || sc->fac_divisor < 0.0f)
        return fail(SI_E_INVALID, "fac_divisor must be finite and >= 0");
    if (sc->kind != SI_SCHED_FAC_PROB && sc->fac_divisor > 0.0f && sc->fac_divisor < 1.0f)
        return fail(SI_E_INVALID, "fac_divisor must be >= 1");
    if (sc->group < 0 || sc->group > kMaxGroup) return fail(SI_E_INVALID, "group must be in [0, 8]");
    if (sc->order != SI_ORDER_SPREAD && sc->order != SI_ORDER_CELL && sc->order != SI_ORDER_GIVEN)
        return fail(SI_E_INVALID, "order must be SI_ORDER_SPREAD, SI_ORDER_CELL or SI_ORDER_GIVEN");
    return SI_OK;
}

// Iterations sorted by the cell of their oriented point, in stream-ordered
// memory released (stream-ordered) by the caller after the launch.
si_status cell_order(const Scene& sc, const int32_t* oriented, int64_t N, hipStream_t s,
                     int32_t** mem_out, const int32_t** perm_out) {
    const int64_t nt = scan_tmp_elems(sc.M);
    const int64_t words = 3 * N + sc.M + (sc.M + 1) + nt;
    int32_t* mem = nullptr;
    SI_HIP(pool_alloc((void**)&mem, sizeof(int32_t) * words, s));
    int32_t* perm = mem;
    int32_t* key = perm + N;
    int32_t* rank = key + N;
    int32_t* counts = rank + N;
    int32_t* starts = counts + sc.M;
    int32_t* tmp = starts + sc.M + 1;
    hipError_t e = launch_cell_order(oriented, N, sc, key, rank, counts, starts, tmp, perm, s);
    if (e != hipSuccess) {
        (void)hipFreeAsync(mem, s);
        return hip_fail(e, "cell order");
    }
    *mem_out = mem;
    *perm_out = perm;
    return SI_OK;
}

int auto_workgroups(DeviceState* st, int max_w2, int group) {
    const auto key = std::make_pair(max_w2, group);
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = st->wg_per_cu.find(key);
        if (it != st->wg_per_cu.end()) per_cu = it->second;
    }
    if (per_cu == 0) {
        per_cu = std::min(8, spin_max_wg_per_cu(max_w2, group));
        std::lock_guard<std::mutex> lk(g_mu);
        st->wg_per_cu[key] = per_cu;
    }
    return std::max(1, st->n_cu * per_cu);
}

}  // namespace si

namespace si {

// Launch state of SI_SCHED_WF / AWF / AF: FAC2's chunk of each batch (by
// value in the launch), and one stream-ordered block holding the AWF / AF
// sums (4 doubles, zero) and the WF weights (n_wg floats).
si_status rule_setup(int kind, int64_t N, int n_wg, const si_sched* sched, LaunchDesc& d,
                     char** mem_out, hipStream_t s) {
    // default floor: a spread unit (8 images); smaller chunks cannot share
    // candidate passes between images, whatever the rule asks
    const int64_t mc = sched->min_chunk > 0 ? sched->min_chunk : kSpreadUnit;
    const double x = sched->fac_divisor > 0.0f ? (double)sched->fac_divisor : 2.0;
    d.rule = kind;
    d.min_chunk = (int32_t)mc;
    d.n_bases = 0;
    for (int64_t R = N; R > 0 && d.n_bases < kMaxBases;) {
        const int64_t c = std::max((int64_t)ceil((double)R / (x * (double)n_wg)), mc);
        d.bases[d.n_bases++] = (int32_t)std::min<int64_t>(c, INT32_MAX);
        R -= std::min(R, c * (int64_t)n_wg);
    }
    // weights: the caller's, else the emulated speeds, else 1; sum n_wg.
    // The host vector is this thread's for the current device, reused once
    // its last upload (recorded on an event of that device) is done.
    struct Upload {
        std::vector<float> w;
        hipEvent_t copied = nullptr;
    };
    static thread_local std::map<int, Upload> uploads;
    int dev = 0;
    SI_HIP(hipGetDevice(&dev));
    Upload& up = uploads[dev];
    std::vector<float>& w = up.w;
    hipEvent_t& w_copied = up.copied;
    if (!w_copied) SI_HIP(hipEventCreateWithFlags(&w_copied, hipEventDisableTiming));
    SI_HIP(hipEventSynchronize(w_copied));
    w.assign(n_wg, 1.0f);
    const std::vector<float>& given = worker_weights();
    if (!given.empty()) {
        for (int k = 0; k < n_wg; ++k) w[k] = given[k % given.size()];
    } else if (d.emu_every > 0 && d.emu_place == SI_EMU_EVERY) {
        for (int k = 0; k < n_wg; ++k)
            if (k % d.emu_every == 0) w[k] = 1.0f / (1.0f + d.emu_extra);
    }
    double sum = 0.0;
    for (float v : w) sum += v;
    for (float& v : w) v = (float)((double)v * (double)n_wg / sum);
    const size_t bytes = 4 * sizeof(double) + sizeof(float) * (size_t)n_wg;
    char* mem = nullptr;
    SI_HIP(pool_alloc((void**)&mem, bytes, s));
    hipError_t e = launch_fill(reinterpret_cast<int32_t*>(mem), 8, 0, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(mem + 4 * sizeof(double), w.data(), sizeof(float) * (size_t)n_wg,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(w_copied, s);
    if (e != hipSuccess) {
        (void)hipFreeAsync(mem, s);
        return hip_fail(e, "worker-sized claims");
    }
    d.adapt = reinterpret_cast<double*>(mem);
    d.weights = reinterpret_cast<const float*>(mem + 4 * sizeof(double));
    *mem_out = mem;
    return SI_OK;
}

}  // namespace si

extern "C" si_status si_generate(const si_scene* scene, const int32_t* oriented_idx, int64_t N,
                                 const si_params* params, const si_sched* sched,
                                 float* images_out, uint32_t* counts_out, si_stats* stats,
                                 void* hip_stream) {
    if (!scene) return fail(SI_E_INVALID, "scene is NULL");
    si_status rc = check_sched(sched);
    if (rc != SI_OK) return rc;
    SpinParams p;
    double R;
    rc = make_params(params, &p, &R);
    if (rc != SI_OK) return rc;
    if (N < 0 || N >= INT32_MAX) return fail(SI_E_INVALID, "N must be in [0, 2^31 - 1)");
    if (N == 0) {
        if (stats) {
            stats->kernel_ms = 0;
            stats->pairs_in_support = stats->pairs_tested = 0;
            stats->sched_used = sched->kind;
            stats->n_wg = stats->n_chunks = stats->n_invalid = stats->n_overflow = 0;
        }
        return SI_OK;
    }
    if (!oriented_idx || !images_out || !counts_out)
        return fail(SI_E_INVALID, "oriented_idx, images_out and counts_out must be non-NULL");
    // the grid keeps a 2e-5 relative margin, so 1e-6 of slack stays conservative
    if (scene->max_radius > 0.0f && R > (double)scene->max_radius * (1.0 + 1e-6))
        return fail(SI_E_INVALID, "support radius of params exceeds the scene's max_support_radius");
    int cur_dev = 0;
    SI_HIP(hipGetDevice(&cur_dev));
    if (cur_dev != scene->device) return fail(SI_E_INVALID, "scene lives on another device");
    hipStream_t s = (hipStream_t)hip_stream;
    rc = refuse_capture(s, "si_generate");
    if (rc != SI_OK) return rc;
    DeviceState* st;
    rc = device_state(&st);
    if (rc != SI_OK) return rc;

    p.reach = scene->max_radius > 0.0f ? (int)floor((double)p.radius / scene->h) + 1 : 0;
    if (p.reach > kSub + 1) return fail(SI_E_INVALID, "support radius too large for the grid");
    const int w2 = p.W * p.W;
    const int group = fit_group(st, sched->group > 0 ? sched->group : default_group(p.W), w2);
    const int n_wg = sched->num_workgroups > 0 ? sched->num_workgroups
                                               : auto_workgroups(st, w2, group);

    LaunchDesc d;
    memset(&d, 0, sizeof(d));
    apply_emulated_workers(d);
    d.single.scene = view_of(*scene);
    d.single.p = p;
    d.single.oriented = oriented_idx;
    d.single.images = images_out;
    d.single.counts = counts_out;
    d.single.N = N;
    d.single.perm = nullptr;
    d.items = nullptr;
    d.group = group;

    int kind = sched->kind;
    Chunk* chunks = nullptr;
    int n_chunks = 0;
    char* learned_mem = nullptr;
    if (kind == SI_SCHED_LEARNED) {
        LearnedPlan plan;
        rc = sched->model ? learned_table(st, scene, oriented_idx, N, params, sched, n_wg, group,
                                          &plan, s)
                          : SI_E_UNSUPPORTED;
        if (rc == SI_E_UNSUPPORTED) {
            if (!sched->fallback_to_fac)
                return fail(SI_E_INVALID, "SI_SCHED_LEARNED needs a model (fallback disabled)");
            kind = SI_SCHED_FAC;  // FAC is the fallback of the learned schedule
        } else if (rc != SI_OK) {
            return rc;
        } else {
            learned_mem = plan.mem;
            d.single.perm = plan.perm;
            chunks = plan.chunks;
            n_chunks = plan.max_chunks;
            d.n_chunks_dev = plan.n_chunks_dev;
        }
    }
    int32_t* order_mem = nullptr;
    char* rule_mem = nullptr;
    void* table_entry = nullptr;
    if (kind >= SI_SCHED_WF) {
        // claims sized by the workgroups: FAC2's batch chunks by value, the
        // WF weights and the AWF / AF sums in one stream-ordered block
        rc = rule_setup(kind, N, n_wg, sched, d, &rule_mem, s);
        if (rc != SI_OK) return rc;
        chunks = nullptr;
        n_chunks = 1;
    }
    if (kind != SI_SCHED_LEARNED) {
        if (kind < SI_SCHED_WF) {
            rc = get_table(st, kind, N, n_wg, sched->min_chunk, sched->fac_divisor, &chunks,
                           &n_chunks, s, &table_entry);
            if (rc != SI_OK) return rc;
        }
        if (sched->order != SI_ORDER_GIVEN && scene->n_cells > 1) {
            rc = cell_order(*scene, oriented_idx, N, s, &order_mem, &d.single.perm);
            if (rc != SI_OK) {
                if (table_entry) (void)table_used(st, table_entry, s, false);
                return rc;
            }
            if (sched->order == SI_ORDER_SPREAD) {
                d.single.spread_full = (int32_t)(N / kSpreadUnit);
                d.single.spread_mult = spread_mult(N / kSpreadUnit);
                if (d.single.spread_mult == 0) d.single.spread_full = 0;
            }
        }
    }
    d.chunks = chunks;
    d.n_chunks = n_chunks;
    d.dynamic = kind == SI_SCHED_STATIC ? 0 : 1;
    rc = run_launch(st, d, n_wg, w2, stats, s, kind);
    if (table_entry) {
        // recorded even after a failed launch: work enqueued before the
        // failure may still read the table
        const si_status r2 = table_used(st, table_entry, s, true);
        if (rc == SI_OK) rc = r2;
    }
    if (order_mem) (void)hipFreeAsync(order_mem, s);
    if (learned_mem) (void)hipFreeAsync(learned_mem, s);
    if (rule_mem) (void)hipFreeAsync(rule_mem, s);
    return rc;
}

extern "C" {

const char* si_status_string(si_status status) {
    switch (status) {
        case SI_OK: return "SI_OK";
        case SI_E_INVALID: return "SI_E_INVALID";
        case SI_E_OOM: return "SI_E_OOM";
        case SI_E_DEVICE: return "SI_E_DEVICE";
        case SI_E_UNSUPPORTED: return "SI_E_UNSUPPORTED";
    }
    return "unknown si_status";
}

const char* si_last_error(void) { return g_last_error.c_str(); }

si_status si_set_emulated_workers(int32_t every, float slowdown) {
    if (every < 0) return fail(SI_E_INVALID, "every must be >= 0");
    if (!isfinite(slowdown) || slowdown < 1.0f) return fail(SI_E_INVALID, "slowdown must be >= 1");
    g_emu_every = slowdown > 1.0f ? every : 0;
    g_emu_slowdown = slowdown;
    return SI_OK;
}

si_status si_set_emulated_mode(int32_t busy, int32_t placement) {
    if (busy != 0 && busy != 1) return fail(SI_E_INVALID, "busy must be 0 or 1");
    if (placement < SI_EMU_EVERY || placement > SI_EMU_LAST)
        return fail(SI_E_INVALID, "placement must be SI_EMU_EVERY, SI_EMU_FIRST or SI_EMU_LAST");
    g_emu_busy = busy;
    g_emu_place = placement;
    return SI_OK;
}

si_status si_set_worker_weights(const float* weights, int32_t n) {
    if (n < 0) return fail(SI_E_INVALID, "n must be >= 0");
    if (n > 0 && !weights) return fail(SI_E_INVALID, "weights is NULL");
    for (int32_t i = 0; i < n; ++i)
        if (!isfinite(weights[i]) || !(weights[i] > 0.0f))
            return fail(SI_E_INVALID, "weights must be positive and finite");
    g_weights.assign(weights, weights + n);
    return SI_OK;
}

int64_t si_rule_wf_chunk(double w, int64_t base, int64_t remaining, int32_t min_chunk) {
    return wf_chunk(w, base, remaining, std::max(1, min_chunk));
}

double si_rule_awf_weight(double rate, double rate_sum, int32_t n_meas, int32_t P) {
    return awf_weight(rate, rate_sum, n_meas, P);
}

int64_t si_rule_af_chunk(double var_over_mu_sum, double inv_mu_sum, int32_t n_meas, int32_t P,
                         int64_t remaining, double mu, int32_t min_chunk) {
    double D, T;
    af_terms(var_over_mu_sum, inv_mu_sum, n_meas, P, &D, &T);
    return af_chunk(D, T, remaining, mu, std::max(1, min_chunk));
}

si_status si_set_kernel_events(void* begin_event, void* end_event) {
    if ((begin_event == nullptr) != (end_event == nullptr))
        return fail(SI_E_INVALID, "give both events or neither");
    g_ev_begin = (hipEvent_t)begin_event;
    g_ev_end = (hipEvent_t)end_event;
    return SI_OK;
}

int32_t si_abi_version(void) { return SI_ABI_VERSION; }

si_status si_device_errors(void* hip_stream) {
    uint32_t seen = 0;
    SI_HIP(take_invalid_flag((hipStream_t)hip_stream, &seen));
    if (seen)
        return fail(SI_E_INVALID,
                    "a generation launch on this device met oriented_idx entries outside [0, M)");
    return SI_OK;
}

}  // extern "C"
