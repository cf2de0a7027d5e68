// Batched generation: the images of many scenes in one persistent launch.
//
// The per-image loops of all items are concatenated into one DOALL loop of
// sum(N) iterations.  A schedule of Section 2.2 is computed over the whole
// concatenation for P workgroups and every chunk that crosses an item
// boundary is split there, so that a chunk never spans two scenes (STATIC
// keeps each workgroup's pieces in its own range).  The cell ordering of the
// iterations is one counting sort over all items (keys offset by each item's
// cell count).  With use_graph the sort and the spin kernel are captured once
// into a HIP graph, cached per item list, and replayed.
//
// A launch sizes its LDS for its largest image, so W <= 32 images sharing a
// launch with W = 64 images would run at that launch's lower occupancy (three
// workgroups per CU instead of five).  Items are therefore launched in two
// classes, W <= 32 and W > 32, one after the other on the stream (one graph
// holds both); each class is its own concatenated loop, scheduled as above.
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "si_internal.h"

namespace si {

namespace {

struct Flat {
    std::vector<Item> items;
    std::vector<int64_t> item_off;   // n + 1
    std::vector<int64_t> key_base;   // n + 1: prefix of the items' scene sizes
    std::vector<Chunk> chunks;
    std::vector<int32_t> wg_first;   // static only, n_wg + 1
    int max_w2 = 0;
    int group = 0;
    int n_wg = 0;
    int kind = 0;
    bool ordered = false;
    int64_t total_N = 0;
    int64_t total_cells = 0;
    int64_t total_keys = 0;
    // SI_SCHED_LEARNED: the plan is computed on the device before each launch
    bool learned = false;
    const si_cost_model* model = nullptr;
    float divisor = 0.0f;
    std::vector<int64_t> unit_off;  // n + 1
    std::vector<float> f11;         // n
    std::vector<int64_t> sat_off;   // 3 (n + 1)
    int64_t sat_pass[3] = {0, 0, 0};
    int64_t n_units = 0;
};

// Device memory of one flattened launch (one allocation).
struct FlatMem {
    char* base = nullptr;
    size_t bytes = 0;
    Item* items = nullptr;
    int64_t* item_off = nullptr;
    int64_t* key_base = nullptr;
    Chunk* chunks = nullptr;
    int32_t* wg_first = nullptr;
    int32_t* perm = nullptr;
    int32_t* key = nullptr;
    int32_t* rank = nullptr;
    int32_t* counts = nullptr;
    int32_t* starts = nullptr;
    int32_t* tmp = nullptr;
    unsigned long long* stats = nullptr;  // 4 + n_wg words
    LearnedMulti lm;                      // learned schedule only
    // host copy of the item table with its device pointers filled in: the
    // source of an asynchronous upload, so it lives as long as this record
    std::vector<Item> host_items;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Lay the buffers out in one block; returns the byte size.
size_t layout(const Flat& f, FlatMem& m, char* base) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + o : nullptr;
        o += align_up(std::max<size_t>(bytes, 1));
        return p;
    };
    const size_t n = f.items.size();
    m.items = (Item*)take(sizeof(Item) * n);
    m.item_off = (int64_t*)take(sizeof(int64_t) * (n + 1));
    m.key_base = (int64_t*)take(sizeof(int64_t) * (n + 1));
    m.chunks = (Chunk*)take(sizeof(Chunk) * f.chunks.size());
    m.wg_first = (int32_t*)take(sizeof(int32_t) * f.wg_first.size());
    m.stats = (unsigned long long*)take(sizeof(unsigned long long) * (4 + (size_t)f.n_wg));
    if (f.ordered) {
        m.perm = (int32_t*)take(sizeof(int32_t) * f.total_N);
        m.key = (int32_t*)take(sizeof(int32_t) * f.total_N);
        m.rank = (int32_t*)take(sizeof(int32_t) * f.total_N);
        m.counts = (int32_t*)take(sizeof(int32_t) * f.total_keys);
        m.starts = (int32_t*)take(sizeof(int32_t) * (f.total_keys + 1));
        m.tmp = (int32_t*)take(sizeof(int32_t) * scan_tmp_elems(f.total_keys));
    }
    if (f.learned) {
        LearnedMulti size_only;
        const int ni = (int)f.items.size();
        char* lb = take(learned_multi_layout(ni, f.total_N, f.n_units, f.n_wg, f.sat_pass,
                                             size_only, nullptr));
        if (base) learned_multi_layout(ni, f.total_N, f.n_units, f.n_wg, f.sat_pass, m.lm, lb);
    }
    m.base = base;
    m.bytes = o;
    return o;
}

void flat_chunks(Flat& f, int min_chunk, float divisor) {
    const int64_t total = f.total_N;
    const int P = f.n_wg;
    const int64_t n = chunk_sizes(f.kind, total, P, min_chunk, divisor, nullptr, 0);
    std::vector<int64_t> st(n + 1);
    chunk_sizes(f.kind, total, P, min_chunk, divisor, st.data(), n + 1);
    const bool stat = f.kind == SI_SCHED_STATIC;
    if (stat) f.wg_first.assign(P + 1, 0);
    size_t it = 0;
    for (int64_t c = 0; c < n; ++c) {
        if (stat) f.wg_first[c] = (int32_t)f.chunks.size();
        int64_t a = st[c];
        const int64_t b = st[c + 1];
        while (a < b) {
            while (f.item_off[it + 1] <= a) ++it;
            const int64_t e = std::min(b, f.item_off[it + 1]);
            f.chunks.push_back({(int32_t)it, (int32_t)(a - f.item_off[it]),
                                (int32_t)(e - f.item_off[it])});
            a = e;
        }
    }
    if (stat) f.wg_first[P] = (int32_t)f.chunks.size();
}

// The flattened launch of items sel[0..] (indices into items).
si_status build_flat(DeviceState* st, const si_batch_item* items, const std::vector<int32_t>& sel,
                     const si_sched* sched, Flat& f) {
    int dev = 0;
    SI_HIP(hipGetDevice(&dev));
    f.item_off.push_back(0);
    f.key_base.push_back(0);
    for (const int32_t k : sel) {
        const si_batch_item& b = items[k];
        if (b.N == 0) continue;
        if (!b.scene) return fail(SI_E_INVALID, "batch item " + std::to_string(k) + ": scene is NULL");
        if (b.N < 0 || b.N >= INT32_MAX)
            return fail(SI_E_INVALID, "batch item " + std::to_string(k) + ": N out of range");
        if (!b.oriented_idx || !b.images_out || !b.counts_out)
            return fail(SI_E_INVALID, "batch item " + std::to_string(k) + ": NULL buffer");
        if (b.scene->device != dev)
            return fail(SI_E_INVALID, "batch item " + std::to_string(k) + ": scene on another device");
        SpinParams p;
        double R;
        si_status rc = make_params(&b.params, &p, &R);
        if (rc != SI_OK) return fail(rc, "batch item " + std::to_string(k) + ": " + si_last_error());
        const Scene& sc = *b.scene;
        if (sc.max_radius > 0.0f && R > (double)sc.max_radius * (1.0 + 1e-6))
            return fail(SI_E_INVALID, "batch item " + std::to_string(k) +
                                          ": support radius exceeds the scene's max_support_radius");
        p.reach = sc.max_radius > 0.0f ? (int)floor((double)p.radius / sc.h) + 1 : 0;
        if (p.reach > kSub + 1) return fail(SI_E_INVALID, "support radius too large for the grid");
        f.f11.push_back((float)(R / (kSub * sc.h)));
        Item it;
        memset(&it, 0, sizeof(it));
        it.scene = view_of(sc);
        it.p = p;
        it.oriented = b.oriented_idx;
        it.images = b.images_out;
        it.counts = b.counts_out;
        it.N = b.N;
        it.perm = nullptr;
        f.items.push_back(it);
        f.item_off.push_back(f.item_off.back() + b.N);
        f.key_base.push_back(f.key_base.back() + sc.M);
        f.total_cells += sc.n_cells;
        f.max_w2 = std::max(f.max_w2, p.W * p.W);
    }
    f.total_N = f.item_off.back();
    f.total_keys = f.key_base.back();
    if (f.total_N >= INT32_MAX || f.total_keys >= INT32_MAX)
        return fail(SI_E_INVALID, "batch too large (2^31 images or scene points)");
    if (f.items.empty()) return SI_OK;
    f.kind = sched->kind;
    if (f.kind == SI_SCHED_LEARNED) {
        if (!sched->model) {
            if (!sched->fallback_to_fac)
                return fail(SI_E_INVALID, "SI_SCHED_LEARNED needs a model (fallback disabled)");
            f.kind = SI_SCHED_FAC;  // FAC is the fallback of the learned schedule
        } else {
            f.learned = true;
            f.model = sched->model;
        }
    }
    int max_W = 2;
    while (max_W * max_W < f.max_w2) ++max_W;
    const int g = sched->group > 0 ? sched->group : default_group(max_W);
    f.group = fit_group(st, g, f.max_w2);
    f.n_wg = sched->num_workgroups > 0 ? sched->num_workgroups
                                       : auto_workgroups(st, f.max_w2, f.group);
    f.ordered = sched->order != SI_ORDER_GIVEN && f.total_cells > (int64_t)f.items.size();
    if (f.ordered && sched->order == SI_ORDER_SPREAD && !f.learned) {
        for (Item& it : f.items) {
            it.spread_mult = spread_mult(it.N / kSpreadUnit);
            it.spread_full = it.spread_mult ? (int32_t)(it.N / kSpreadUnit) : 0;
        }
    }
    if (f.learned) {
        if (f.n_wg > kMaxLearnedP)
            return fail(SI_E_INVALID, "the learned schedule supports at most " +
                                          std::to_string(kMaxLearnedP) + " workgroups");
        std::vector<int64_t> Ns;
        for (const Item& it : f.items) Ns.push_back(it.N);
        f.unit_off.resize(f.items.size() + 1);
        f.n_units = learned_units(Ns.data(), (int)Ns.size(), f.unit_off.data());
        f.sat_off.resize(3 * (f.items.size() + 1));
        const size_t n1 = f.items.size() + 1;
        sat_offsets(f.items.data(), (int)f.items.size(), f.sat_off.data());
        for (int k = 0; k < 3; ++k) f.sat_pass[k] = f.sat_off[(k + 1) * n1 - 1];
        f.divisor = sched->fac_divisor;
    } else {
        // FAC's default ratio: x = 2 (FAC2) assumes iterations of similar
        // cost, as in one spread-ordered scene.  A concatenation of several
        // scenes (other widths, densities and sizes) varies much more, and
        // factoring's batch ratio grows with the cost variation; a larger
        // ratio also makes the first batches cover fewer items, so the
        // workgroups running at once share fewer scenes in the L2.  A launch
        // over several items takes x = 12 and chunks of at least 16 images
        // unless the caller sets them.
        const bool multi = f.kind == SI_SCHED_FAC && f.items.size() > 1;
        const float dv = sched->fac_divisor > 0.0f ? sched->fac_divisor : multi ? 12.0f : 0.0f;
        const int mc = sched->min_chunk > 0 ? sched->min_chunk : multi ? 16 : 0;
        flat_chunks(f, mc, dv);
    }
    return SI_OK;
}

// Image-size class of a batch item (see the file comment).
int size_class(const si_batch_item& b) { return b.params.W > 32 ? 1 : 0; }
constexpr int kClasses = 2;

// The flattened launches of a batch, one per non-empty class, in class order.
si_status build_launches(DeviceState* st, const si_batch_item* items, int32_t n_items,
                         const si_sched* sched, std::vector<Flat>& flats) {
    std::vector<int32_t> sel[kClasses];
    for (int32_t k = 0; k < n_items; ++k)
        if (items[k].N != 0) sel[size_class(items[k])].push_back(k);
    flats.clear();
    for (int c = 0; c < kClasses; ++c) {
        if (sel[c].empty()) continue;
        Flat f;
        const si_status rc = build_flat(st, items, sel[c], sched, f);
        if (rc != SI_OK) return rc;
        if (!f.items.empty()) flats.push_back(std::move(f));
    }
    return SI_OK;
}

// Upload the host-side tables into m, on s; the caller synchronises s before
// f's tables go (the item table's staged copy lives in m).
si_status upload(const Flat& f, FlatMem& m, hipStream_t s) {
    std::vector<Item>& items = m.host_items;
    items = f.items;
    for (size_t i = 0; i < items.size(); ++i)
        items[i].perm = f.learned   ? m.lm.perm + f.item_off[i]
                        : f.ordered ? m.perm + f.item_off[i]
                                    : nullptr;
    SI_HIP(hipMemcpyAsync(m.items, items.data(), sizeof(Item) * items.size(),
                          hipMemcpyHostToDevice, s));
    SI_HIP(hipMemcpyAsync(m.item_off, f.item_off.data(), sizeof(int64_t) * f.item_off.size(),
                          hipMemcpyHostToDevice, s));
    SI_HIP(hipMemcpyAsync(m.key_base, f.key_base.data(), sizeof(int64_t) * f.key_base.size(),
                          hipMemcpyHostToDevice, s));
    if (!f.chunks.empty())
        SI_HIP(hipMemcpyAsync(m.chunks, f.chunks.data(), sizeof(Chunk) * f.chunks.size(),
                              hipMemcpyHostToDevice, s));
    if (f.learned) {
        SI_HIP(hipMemcpyAsync(m.lm.unit_off, f.unit_off.data(), sizeof(int64_t) * f.unit_off.size(),
                              hipMemcpyHostToDevice, s));
        SI_HIP(hipMemcpyAsync(m.lm.f11, f.f11.data(), sizeof(float) * f.f11.size(),
                              hipMemcpyHostToDevice, s));
        SI_HIP(hipMemcpyAsync(m.lm.sat_off, f.sat_off.data(), sizeof(int64_t) * f.sat_off.size(),
                              hipMemcpyHostToDevice, s));
    }
    if (!f.wg_first.empty())
        SI_HIP(hipMemcpyAsync(m.wg_first, f.wg_first.data(), sizeof(int32_t) * f.wg_first.size(),
                              hipMemcpyHostToDevice, s));
    return SI_OK;
}

LaunchDesc desc_of(const Flat& f, const FlatMem& m, uint32_t* counter, bool stats) {
    LaunchDesc d;
    memset(&d, 0, sizeof(d));
    apply_emulated_workers(d);
    d.items = m.items;
    d.chunks = m.chunks;
    d.n_chunks = (int32_t)f.chunks.size();
    if (f.learned) {
        d.chunks = m.lm.chunks;
        d.n_chunks = (int32_t)f.n_units;  // capacity; the count is on the device
        d.n_chunks_dev = m.lm.n_chunks;
    }
    d.dynamic = f.kind == SI_SCHED_STATIC ? 0 : 1;
    d.wg_first = f.kind == SI_SCHED_STATIC ? m.wg_first : nullptr;
    d.counter = counter;
    d.group = f.group;
    d.max_w2 = f.max_w2;
    d.ovf_limit = 65536u;
    if (const char* lim = getenv("SI_TEST_OVERFLOW_LIMIT")) d.ovf_limit = (uint32_t)atol(lim);
    if (stats) {
        d.stat_tested = m.stats;
        d.stat_support = m.stats + 1;
        d.stat_invalid = reinterpret_cast<uint32_t*>(m.stats + 2);
        d.stat_overflow = reinterpret_cast<uint32_t*>(m.stats + 3);
        d.wg_ns = m.stats + 4;
    }
    return d;
}

// Enqueue ordering (+ learned plan) + spin kernel (the body of a graph, or a
// direct launch).  ev0/ev1 and ub/ue bracket the spin kernel.
hipError_t enqueue(const Flat& f, const FlatMem& m, const LaunchDesc& d, bool stats,
                   hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ub, hipEvent_t ue, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (stats) e = launch_fill(reinterpret_cast<int32_t*>(m.stats), 2 * (4 + (int64_t)f.n_wg), 0, s);
    if (e == hipSuccess && f.ordered)
        e = launch_cell_order_multi(m.items, m.item_off, m.key_base, (int)f.items.size(),
                                    f.total_N, f.total_keys, m.key, m.rank, m.counts, m.starts,
                                    m.tmp, m.perm, s);
    if (e == hipSuccess && f.learned)
        e = learned_multi_enqueue(f.model, m.lm, m.items, m.item_off, (int)f.items.size(),
                                  f.ordered ? m.perm : nullptr, f.total_N, f.n_units, f.n_wg,
                                  f.divisor, s);
    if (e == hipSuccess && ev0) e = hipEventRecord(ev0, s);
    if (e == hipSuccess && ub) e = hipEventRecord(ub, s);
    if (e == hipSuccess) e = launch_spin(d, f.n_wg, s);
    if (e == hipSuccess && ue) e = hipEventRecord(ue, s);
    if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
    return e;
}

// Statistics of the launches of one call, summed over them; kernel_ms is the
// time from the first spin launch to the end of the last.  n_wg and the
// per-workgroup busy times are those of the largest launch's workgroup
// slots (busy times summed over the launches).
si_status read_stats(DeviceState* st, const std::vector<Flat>& flats,
                     const std::vector<FlatMem>& mems, float ms, si_stats* stats, hipStream_t s) {
    stats->kernel_ms = ms;
    stats->pairs_tested = stats->pairs_in_support = 0;
    stats->n_invalid = stats->n_overflow = 0;
    stats->sched_used = flats.empty() ? 0 : flats[0].kind;
    stats->n_wg = 0;
    stats->n_chunks = 0;
    for (const Flat& f : flats) stats->n_wg = std::max(stats->n_wg, f.n_wg);
    std::vector<uint64_t> busy((size_t)stats->n_wg, 0);
    for (size_t c = 0; c < flats.size(); ++c) {
        const Flat& f = flats[c];
        const FlatMem& m = mems[c];
        std::vector<unsigned long long> h(4 + (size_t)f.n_wg);
        SI_HIP(hipMemcpyAsync(h.data(), m.stats, sizeof(unsigned long long) * h.size(),
                              hipMemcpyDeviceToHost, s));
        SI_HIP(hipStreamSynchronize(s));
        stats->pairs_tested += h[0];
        stats->pairs_in_support += h[1];
        stats->n_invalid += (int32_t)(uint32_t)h[2];
        stats->n_overflow += (int32_t)(uint32_t)h[3];
        if (f.learned) {
            int32_t nc = 0;
            SI_HIP(hipMemcpy(&nc, m.lm.n_chunks, sizeof(nc), hipMemcpyDeviceToHost));
            stats->n_chunks += nc;
        } else {
            stats->n_chunks += (int32_t)f.chunks.size();
        }
        for (int i = 0; i < f.n_wg; ++i)
            busy[i] += (uint64_t)((double)h[4 + i] * 1e6 / (double)st->wall_khz);
    }
    if (stats->wg_busy_ns) {
        const int n = std::min(stats->wg_busy_cap, stats->n_wg);
        for (int i = 0; i < n; ++i) stats->wg_busy_ns[i] = busy[i];
    }
    if (stats->n_invalid) return fail(SI_E_INVALID, "oriented_idx holds indices outside [0, M)");
    return SI_OK;
}

// ---- graph cache ----
struct GraphEntry {
    std::vector<Flat> flats;  // one launch per image-size class
    std::vector<FlatMem> mems;
    std::vector<uint32_t*> counters;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    uint64_t last_use = 0;
    std::vector<uint64_t> serials;  // scenes and cost model the graph reads
};

std::mutex g_graph_mu;
std::map<std::string, GraphEntry*> g_graphs;
uint64_t g_graph_clock = 0;
constexpr size_t kMaxGraphs = 8;

void free_entry(GraphEntry* e) {
    if (!e) return;
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->ev0) (void)hipEventDestroy(e->ev0);
    if (e->ev1) (void)hipEventDestroy(e->ev1);
    for (FlatMem& m : e->mems) (void)hipFree(m.base);
    for (uint32_t* c : e->counters) (void)hipFree(c);
    delete e;
}

}  // namespace

void drop_graphs_of(uint64_t serial) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    bool synced = false;
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
        const std::vector<uint64_t>& v = it->second->serials;
        if (std::find(v.begin(), v.end(), serial) == v.end()) {
            ++it;
            continue;
        }
        if (!synced) {  // a replay may still be queued
            (void)hipDeviceSynchronize();
            synced = true;
        }
        free_entry(it->second);
        it = g_graphs.erase(it);
    }
}

namespace {

std::string graph_key(const si_batch_item* items, int32_t n_items, const si_sched* sched,
                      bool stats, int dev) {
    std::string k;
    k.reserve(64 + (size_t)n_items * 96);
    auto put = [&](const void* p, size_t n) { k.append((const char*)p, n); };
    put(&dev, sizeof(dev));
    put(&stats, sizeof(stats));
    si_sched sc = *sched;
    put(&sc.kind, sizeof(sc.kind));
    put(&sc.num_workgroups, sizeof(sc.num_workgroups));
    put(&sc.min_chunk, sizeof(sc.min_chunk));
    put(&sc.fac_divisor, sizeof(sc.fac_divisor));
    put(&sc.group, sizeof(sc.group));
    put(&sc.order, sizeof(sc.order));
    // objects by serial, not by address: a freed scene's or model's handle
    // and device memory can be handed out again to a new one
    const uint64_t mser = model_serial(sc.model);
    put(&mser, sizeof(mser));
    put(&sc.fallback_to_fac, sizeof(sc.fallback_to_fac));
    const char* lim = getenv("SI_TEST_OVERFLOW_LIMIT");
    k.append(lim ? lim : "-");
    LaunchDesc emu;  // the calling thread's emulated-worker setting
    memset(&emu, 0, sizeof(emu));
    apply_emulated_workers(emu);
    put(&emu.emu_every, sizeof(emu.emu_every));
    put(&emu.emu_extra, sizeof(emu.emu_extra));
    for (int32_t i = 0; i < n_items; ++i) {
        const si_batch_item& b = items[i];
        const uint64_t ser = b.scene ? b.scene->serial : 0;
        put(&ser, sizeof(ser));
        put(&b.oriented_idx, sizeof(b.oriented_idx));
        put(&b.N, sizeof(b.N));
        put(&b.params, sizeof(b.params));
        put(&b.images_out, sizeof(b.images_out));
        put(&b.counts_out, sizeof(b.counts_out));
    }
    return k;
}

si_status make_graph(DeviceState* st, const si_batch_item* items, int32_t n_items,
                     const si_sched* sched, bool stats, GraphEntry** out) {
    GraphEntry* e = new (std::nothrow) GraphEntry();
    if (!e) return fail(SI_E_OOM, "host allocation failed");
    si_status rc = build_launches(st, items, n_items, sched, e->flats);
    if (rc != SI_OK) { delete e; return rc; }
    if (e->flats.empty()) {  // nothing to launch: an entry without a graph
        *out = e;
        return SI_OK;
    }
    const size_t nl = e->flats.size();
    e->mems.resize(nl);
    e->counters.assign(nl, nullptr);
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipError_t err = hipSuccess;
    for (size_t c = 0; c < nl && err == hipSuccess; ++c) {
        char* base = nullptr;
        err = hipMalloc(&base, layout(e->flats[c], e->mems[c], nullptr));
        if (err == hipSuccess) layout(e->flats[c], e->mems[c], base);
        if (err == hipSuccess) err = hipMalloc(&e->counters[c], 2 * sizeof(uint32_t));
        if (err == hipSuccess) err = hipMemset(e->counters[c], 0, 2 * sizeof(uint32_t));
    }
    if (err == hipSuccess) err = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (err != hipSuccess) {
        free_entry(e);
        return hip_fail(err, "graph setup");
    }
    for (size_t c = 0; c < nl && rc == SI_OK; ++c) rc = upload(e->flats[c], e->mems[c], cs);
    if (rc == SI_OK) {
        err = hipStreamSynchronize(cs);
        if (err == hipSuccess) err = hipEventCreate(&e->ev0);
        if (err == hipSuccess) err = hipEventCreate(&e->ev1);
        if (err == hipSuccess) err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (err == hipSuccess) {
            hipError_t qe = hipSuccess;
            for (size_t c = 0; c < nl && qe == hipSuccess; ++c) {
                const LaunchDesc d = desc_of(e->flats[c], e->mems[c], e->counters[c], stats);
                qe = enqueue(e->flats[c], e->mems[c], d, stats, nullptr, nullptr, nullptr, nullptr,
                             cs);
            }
            err = hipStreamEndCapture(cs, &graph);
            if (qe != hipSuccess) err = qe;
        }
        if (err == hipSuccess) err = hipGraphInstantiate(&e->exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (err != hipSuccess) rc = hip_fail(err, "graph capture");
    }
    (void)hipStreamDestroy(cs);
    if (rc != SI_OK) {
        free_entry(e);
        return rc;
    }
    *out = e;
    return SI_OK;
}

}  // namespace

}  // namespace si

using namespace si;

extern "C" si_status si_generate_batched(const si_batch_item* items, int32_t n_items,
                                         const si_sched* sched, int32_t use_graph,
                                         si_stats* stats, void* hip_stream) {
    if (n_items < 0 || (n_items > 0 && !items)) return fail(SI_E_INVALID, "bad item list");
    si_status rc = check_sched(sched);
    if (rc == SI_OK && sched->kind >= SI_SCHED_WF)
        return fail(SI_E_UNSUPPORTED, "SI_SCHED_WF, AWF and AF run in si_generate only");
    if (rc != SI_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    rc = refuse_capture(s, "si_generate_batched");
    if (rc != SI_OK) return rc;
    DeviceState* st;
    rc = device_state(&st);
    if (rc != SI_OK) return rc;
    hipEvent_t ub = nullptr, ue = nullptr;
    user_kernel_events(&ub, &ue);

    if (!use_graph) {
        std::vector<Flat> flats;
        rc = build_launches(st, items, n_items, sched, flats);
        if (rc != SI_OK) return rc;
        if (flats.empty()) {
            if (stats) memset(stats, 0, offsetof(si_stats, wg_busy_cap));
            return SI_OK;
        }
        const size_t nl = flats.size();
        std::vector<FlatMem> mems(nl);
        std::vector<char*> bases(nl, nullptr);
        for (size_t c = 0; c < nl && rc == SI_OK; ++c) {
            const hipError_t e = pool_alloc((void**)&bases[c], layout(flats[c], mems[c], nullptr), s);
            if (e != hipSuccess) {
                rc = hip_fail(e, "batched launch tables");
                break;
            }
            layout(flats[c], mems[c], bases[c]);
            rc = upload(flats[c], mems[c], s);
        }
        // the staged host tables are about to go out of scope
        if (rc == SI_OK && hipStreamSynchronize(s) != hipSuccess)
            rc = fail(SI_E_DEVICE, "stream synchronisation failed");
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (rc == SI_OK && stats) {
            if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
                rc = fail(SI_E_DEVICE, "event creation failed");
        }
        for (size_t c = 0; c < nl && rc == SI_OK; ++c) {
            // events bracket the spin launches: from the first to the last
            const bool first = c == 0, last = c + 1 == nl;
            LaunchDesc d = desc_of(flats[c], mems[c], take_counter(st), stats != nullptr);
            hipError_t e = enqueue(flats[c], mems[c], d, stats != nullptr, first ? e0 : nullptr,
                                   last ? e1 : nullptr, first ? ub : nullptr, last ? ue : nullptr,
                                   s);
            if (e != hipSuccess) rc = hip_fail(e, "batched launch");
        }
        if (rc == SI_OK && stats) {
            float ms = 0.0f;
            (void)hipEventSynchronize(e1);
            (void)hipEventElapsedTime(&ms, e0, e1);
            rc = read_stats(st, flats, mems, ms, stats, s);
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (char* b : bases)
            if (b) (void)hipFreeAsync(b, s);
        return rc;
    }

    // ---- graph mode ----
    int dev = 0;
    SI_HIP(hipGetDevice(&dev));
    const std::string key = graph_key(items, n_items, sched, stats != nullptr, dev);
    GraphEntry* e = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        auto it = g_graphs.find(key);
        if (it != g_graphs.end()) e = it->second;
    }
    if (!e) {
        rc = make_graph(st, items, n_items, sched, stats != nullptr, &e);
        if (rc != SI_OK) return rc;
        for (int32_t i = 0; i < n_items; ++i)
            if (items[i].scene) e->serials.push_back(items[i].scene->serial);
        if (sched->model) e->serials.push_back(model_serial(sched->model));
        std::lock_guard<std::mutex> lk(g_graph_mu);
        auto again = g_graphs.find(key);
        if (again != g_graphs.end()) {  // another thread captured the same list meanwhile
            (void)hipDeviceSynchronize();
            free_entry(e);
            e = again->second;
        } else if (g_graphs.size() >= kMaxGraphs) {  // evict the least recently used entry
            auto victim = g_graphs.begin();
            for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
                if (it->second->last_use < victim->second->last_use) victim = it;
            (void)hipDeviceSynchronize();
            free_entry(victim->second);
            g_graphs.erase(victim);
        }
        if (again == g_graphs.end()) g_graphs[key] = e;
    }
    e->last_use = ++g_graph_clock;
    if (e->flats.empty()) {
        if (stats) memset(stats, 0, offsetof(si_stats, wg_busy_cap));
        return SI_OK;
    }
    if (stats) SI_HIP(hipEventRecord(e->ev0, s));
    if (ub) SI_HIP(hipEventRecord(ub, s));
    SI_HIP(hipGraphLaunch(e->exec, s));
    if (ue) SI_HIP(hipEventRecord(ue, s));
    if (!stats) return SI_OK;
    SI_HIP(hipEventRecord(e->ev1, s));
    SI_HIP(hipEventSynchronize(e->ev1));
    float ms = 0.0f;
    SI_HIP(hipEventElapsedTime(&ms, e->ev0, e->ev1));
    return read_stats(st, e->flats, e->mems, ms, stats, s);
}

// Features of every image of many scenes in one pass of launches (the
// batched learned planner's kernels, in item order).
extern "C" si_status si_features_batched(const si_batch_item* items, int32_t n_items,
                                         float* feats_out, void* hip_stream) {
    if (n_items < 0 || (n_items > 0 && !items)) return fail(SI_E_INVALID, "bad item list");
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<Item> its;
    std::vector<int64_t> off(1, 0);
    std::vector<float> f11;
    for (int32_t k = 0; k < n_items; ++k) {
        const si_batch_item& b = items[k];
        if (b.N == 0) continue;
        if (!b.scene || !b.oriented_idx || b.N < 0 || b.N >= INT32_MAX)
            return fail(SI_E_INVALID, "batch item " + std::to_string(k) + ": bad scene, indices or N");
        SpinParams p;
        double R;
        si_status rc = make_params(&b.params, &p, &R);
        if (rc != SI_OK) return rc;
        Item it;
        memset(&it, 0, sizeof(it));
        it.scene = view_of(*b.scene);
        it.oriented = b.oriented_idx;
        it.N = b.N;
        its.push_back(it);
        off.push_back(off.back() + b.N);
        f11.push_back((float)(R / (kSub * b.scene->h)));
    }
    const int n = (int)its.size();
    const int64_t total = off.back();
    if (total == 0) return SI_OK;
    if (!feats_out) return fail(SI_E_INVALID, "feats_out is NULL");
    if (total >= INT32_MAX) return fail(SI_E_INVALID, "too many images");
    std::vector<int64_t> sat_off(3 * (n + 1));
    const int64_t sat_total = sat_offsets(its.data(), n, sat_off.data());
    const int64_t pass_n[3] = {sat_off[n], sat_off[2 * n + 1], sat_off[3 * n + 2]};
    auto rup = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_it = rup(sizeof(Item) * n), b_off = rup(sizeof(int64_t) * (n + 1));
    const size_t b_f = rup(sizeof(float) * n), b_so = rup(sizeof(int64_t) * sat_off.size());
    char* mem = nullptr;
    SI_HIP(pool_alloc((void**)&mem, b_it + b_off + b_f + b_so + sizeof(int32_t) * sat_total, s));
    Item* d_it = reinterpret_cast<Item*>(mem);
    int64_t* d_off = reinterpret_cast<int64_t*>(mem + b_it);
    float* d_f11 = reinterpret_cast<float*>(mem + b_it + b_off);
    int64_t* d_so = reinterpret_cast<int64_t*>(mem + b_it + b_off + b_f);
    int32_t* d_sat = reinterpret_cast<int32_t*>(mem + b_it + b_off + b_f + b_so);
    hipError_t e = hipMemcpyAsync(d_it, its.data(), sizeof(Item) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_f11, f11.data(), sizeof(float) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_so, sat_off.data(), sizeof(int64_t) * sat_off.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_features_multi(d_it, d_off, n, nullptr, d_f11, d_so, d_sat, pass_n, total,
                                  feats_out, s);
    // the host tables are staged from pageable memory: wait before they go
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(mem, s);
    if (e != hipSuccess) return hip_fail(e, "batched features");
    return SI_OK;
}
