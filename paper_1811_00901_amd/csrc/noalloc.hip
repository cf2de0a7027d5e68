// si_generate_noalloc: spin-image generation that allocates no memory, for
// callers that cannot allocate (tight serving loops, harnesses that forbid
// it).  It is not for stream capture: a capturing stream is refused.
//
// It runs the same kernels as si_generate (Section 2.1, Algorithm 1 per
// image; the chunks of Section 2.2 claimed through one counter).  What
// si_generate allocates per call -- the claim counter, the chunk table and
// the temporaries of the cell-sorted loop order -- lives here in one
// file-scope device array, `scratch`, of SI_NOALLOC_SCRATCH_BYTES: each
// device holds its own copy from the moment the library's code is loaded
// until the process ends.  Every call on a device reuses that device's copy,
// so calls that overlap on one device (two streams, two threads) race on it.
//
// Layout of the scratch array (256-byte aligned regions):
//   [0, 256)            claim counter (2 words), cleared by each call
//   chunk table         n_chunks x {item, start, end}
//   order temporaries   perm (N), key (N), rank (N), counts (M),
//                       starts (M + 1), scan temporaries
#include "si_internal.h"

#include <math.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

// One copy per device; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[SI_NOALLOC_SCRATCH_BYTES];

namespace si {
namespace {

std::mutex g_mu;
std::map<int, char*> g_scratch;  // device -> address of its scratch array

// Set-up, once per device, with that device current.
si_status scratch_of_device(char** out) {
    int dev = 0;
    SI_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        it = g_scratch.emplace(dev, static_cast<char*>(p)).first;
    }
    *out = it->second;
    return SI_OK;
}

size_t rup256(size_t b) { return (b + 255) & ~(size_t)255; }

// Host copies of this thread's last chunk tables on each device, in a ring
// of kRing: a call reuses the oldest once the upload recorded on its event
// (an event of that device) is done, so up to kRing calls can be queued
// before the host waits.  Their storage is kept between calls.
constexpr int kRing = 4;
struct HostRing {
    std::vector<Chunk> table[kRing];
    hipEvent_t copied[kRing] = {};
    int next = 0;
};
thread_local std::vector<int64_t> t_starts;
thread_local std::map<int, HostRing> t_rings;  // device -> ring

}  // namespace
}  // namespace si

using namespace si;

extern "C" si_status si_generate_noalloc(const si_scene* scene, const int32_t* oriented_idx,
                                         int64_t N, const si_params* params,
                                         const si_sched* sched, float* images_out,
                                         uint32_t* counts_out, void* hip_stream) {
    if (!scene) return fail(SI_E_INVALID, "scene is NULL");
    si_status rc = check_sched(sched);
    if (rc != SI_OK) return rc;
    if (sched->kind >= SI_SCHED_WF)
        return fail(SI_E_UNSUPPORTED, "SI_SCHED_WF, AWF and AF run in si_generate only");
    if (sched->kind == SI_SCHED_LEARNED)
        return fail(SI_E_UNSUPPORTED,
                    "si_generate_noalloc runs the fixed schedules only; the learned plan "
                    "needs memory of its own (use si_generate)");
    SpinParams p;
    double R;
    rc = make_params(params, &p, &R);
    if (rc != SI_OK) return rc;
    if (N < 0 || N >= INT32_MAX) return fail(SI_E_INVALID, "N must be in [0, 2^31 - 1)");
    if (N == 0) return SI_OK;
    if (!oriented_idx || !images_out || !counts_out)
        return fail(SI_E_INVALID, "oriented_idx, images_out and counts_out must be non-NULL");
    if (scene->max_radius > 0.0f && R > (double)scene->max_radius * (1.0 + 1e-6))
        return fail(SI_E_INVALID, "support radius of params exceeds the scene's max_support_radius");
    int cur_dev = 0;
    SI_HIP(hipGetDevice(&cur_dev));
    if (cur_dev != scene->device) return fail(SI_E_INVALID, "scene lives on another device");
    hipStream_t s = (hipStream_t)hip_stream;
    // a captured copy would read the host table at every replay, from storage
    // that later calls refill
    rc = refuse_capture(s, "si_generate_noalloc");
    if (rc != SI_OK) return rc;
    DeviceState* st;
    rc = device_state(&st);  // attributes only: allocates nothing
    if (rc != SI_OK) return rc;
    char* base = nullptr;
    rc = scratch_of_device(&base);
    if (rc != SI_OK) return rc;

    p.reach = scene->max_radius > 0.0f ? (int)floor((double)p.radius / scene->h) + 1 : 0;
    if (p.reach > kSub + 1) return fail(SI_E_INVALID, "support radius too large for the grid");
    const int w2 = p.W * p.W;
    const int group = fit_group(st, sched->group > 0 ? sched->group : default_group(p.W), w2);
    const int n_wg = sched->num_workgroups > 0 ? sched->num_workgroups
                                               : auto_workgroups(st, w2, group);

    // ---- what the call needs of the scratch array ----
    const int kind = sched->kind;
    const float dv = kind == SI_SCHED_FAC_PROB ? sched->fac_divisor
                     : sched->fac_divisor > 0.0f ? sched->fac_divisor : 2.0f;
    const int64_t n_chunks = chunk_sizes(kind, N, n_wg, sched->min_chunk, dv, nullptr, 0);
    const bool ordered = sched->order != SI_ORDER_GIVEN && scene->n_cells > 1;
    const int64_t M = scene->M;
    const int64_t order_words = ordered ? 3 * N + M + (M + 1) + scan_tmp_elems(M) : 0;
    const size_t off_table = 256;
    const size_t off_order = off_table + rup256(sizeof(Chunk) * (size_t)n_chunks);
    const size_t need = off_order + rup256(sizeof(int32_t) * (size_t)order_words);
    if (n_chunks > INT32_MAX || need > (size_t)SI_NOALLOC_SCRATCH_BYTES)
        return fail(SI_E_INVALID,
                    "si_generate_noalloc: this call needs " + std::to_string(need) +
                        " bytes of scratch (" + std::to_string(n_chunks) +
                        " chunks" + (ordered ? ", the cell order of N and M points" : "") +
                        "), more than the " + std::to_string((size_t)SI_NOALLOC_SCRATCH_BYTES) +
                        " it has");

    // ---- chunk table (host), in the oldest ring slot once its upload is done ----
    HostRing& ring = t_rings[cur_dev];
    const int slot = ring.next;
    ring.next = (ring.next + 1) % kRing;
    hipEvent_t& copied = ring.copied[slot];
    if (!copied) SI_HIP(hipEventCreateWithFlags(&copied, hipEventDisableTiming));
    SI_HIP(hipEventSynchronize(copied));
    std::vector<Chunk>& host_table = ring.table[slot];
    t_starts.resize((size_t)n_chunks + 1);
    chunk_sizes(kind, N, n_wg, sched->min_chunk, dv, t_starts.data(), n_chunks + 1);
    host_table.resize((size_t)n_chunks);
    for (int64_t i = 0; i < n_chunks; ++i) {
        host_table[i].item = 0;
        host_table[i].start = (int32_t)t_starts[i];
        host_table[i].end = (int32_t)t_starts[i + 1];
    }

    uint32_t* counter = reinterpret_cast<uint32_t*>(base);
    Chunk* table = reinterpret_cast<Chunk*>(base + off_table);
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
    d.chunks = table;
    d.n_chunks = (int32_t)n_chunks;
    d.dynamic = kind == SI_SCHED_STATIC ? 0 : 1;
    d.counter = counter;
    d.max_w2 = w2;
    d.ovf_limit = 65536u;
    if (const char* lim = getenv("SI_TEST_OVERFLOW_LIMIT")) d.ovf_limit = (uint32_t)atol(lim);

    // ---- enqueue: clear the counter, upload the table, order, launch ----
    hipError_t e = launch_fill(reinterpret_cast<int32_t*>(counter), 2, 0, s);
    // the table comes from this thread's ring slot; the call that reuses the
    // slot waits for this event first
    if (e == hipSuccess)
        e = hipMemcpyAsync(table, host_table.data(), sizeof(Chunk) * (size_t)n_chunks,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(copied, s);
    if (e == hipSuccess && ordered) {
        int32_t* perm = reinterpret_cast<int32_t*>(base + off_order);
        int32_t* key = perm + N;
        int32_t* rank = key + N;
        int32_t* counts = rank + N;
        int32_t* starts = counts + M;
        int32_t* tmp = starts + M + 1;
        e = launch_cell_order(oriented_idx, N, *scene, key, rank, counts, starts, tmp, perm, s);
        d.single.perm = perm;
        if (sched->order == SI_ORDER_SPREAD) {
            d.single.spread_full = (int32_t)(N / kSpreadUnit);
            d.single.spread_mult = spread_mult(N / kSpreadUnit);
            if (d.single.spread_mult == 0) d.single.spread_full = 0;
        }
    }
    if (e == hipSuccess) {
        hipEvent_t ev_begin, ev_end;
        user_kernel_events(&ev_begin, &ev_end);
        if (ev_begin) e = hipEventRecord(ev_begin, s);
        if (e == hipSuccess) e = launch_spin(d, n_wg, s);
        if (e == hipSuccess && ev_end) e = hipEventRecord(ev_end, s);
    }
    if (e != hipSuccess) return hip_fail(e, "si_generate_noalloc");
    return SI_OK;
}
