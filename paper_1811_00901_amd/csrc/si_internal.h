// Internal declarations shared by the host runtime and the HIP kernels of
// the spin-image library.  Nothing here is part of the C ABI (include/si.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/si.h"

namespace si {

// ---------------------------------------------------------------- errors --
void set_error(const std::string& msg);
si_status fail(si_status st, const std::string& msg);
si_status hip_fail(hipError_t e, const char* what);
// SI_E_UNSUPPORTED when s is capturing (`what` names the entry point)
si_status refuse_capture(hipStream_t s, const char* what);

#define SI_HIP(call)                                         \
    do {                                                     \
        hipError_t _e = (call);                              \
        if (_e != hipSuccess) return ::si::hip_fail(_e, #call); \
    } while (0)

// ----------------------------------------------------------------- scene --
// Process-wide serial numbers of scenes and cost models, never reused: a
// freed object's address (host handle, pool memory) can come back for the
// next one, its serial cannot, so caches keyed on serials never match a
// later object.
inline uint64_t next_serial() {
    static std::atomic<uint64_t> counter{0};
    return ++counter;
}
// Drop every cached batched-launch graph that was built for the scene or
// cost model of this serial (called when the object is freed).
void drop_graphs_of(uint64_t serial);
// The serial of a cost model (0 for NULL).
uint64_t model_serial(const si_cost_model* m);

// Grid cells per support radius: cell edge h = R_max (1 + 2e-5) / kSub (odd,
// so that the 3 x 3 x 3 coarse cells of the cost features are centred).
constexpr int kSub = 3;
// Points of a cell are sorted by the quarter of the cell their x falls in:
// key = cell * kSubX + floor(kSubX * frac(x / h)), so that a row's candidate
// run can be cut at quarter-cell resolution.
constexpr int kSubX = 4;
// Iterations per unit of the spread cell order (a power of two).
constexpr int kSpreadUnit = 8;
// Cap on the number of grid cells of one scene; a larger box gets bigger cells.
constexpr int64_t kMaxCells = int64_t(1) << 25;

struct Scene {
    uint64_t serial = next_serial();
    int64_t M = 0;
    float4* pos = nullptr;       // sorted by cell: (x, y, z, bits(cell id))
    float4* nrm = nullptr;       // sorted by cell: (nx, ny, nz, bits(original index))
    int32_t* sub_start = nullptr;   // n_cells * kSubX + 1: first point of each key
    int32_t* inv = nullptr;      // original index -> sorted position
    int32_t dims[3] = {1, 1, 1};
    float origin[3] = {0, 0, 0};
    double h = 0;                // cell edge (double, as used to bin the points)
    float max_radius = 0;        // <= 0: brute force, single cell
    int64_t n_cells = 1;
    int device = 0;
    void* mem = nullptr;         // one pool allocation holding the four arrays
};

// --------------------------------------------------------------- kernels --
// Spin-image launch description (passed by value to the kernel).
struct SpinParams {
    int32_t W;
    int32_t mode;            // SI_BIN_*
    float half;              // W / 2
    float inv_bin;           // 1 / B (float of the double quotient)
    float beta_lo, beta_hi;  // extent in beta (mode dependent, see kernel)
    float alpha2_max;        // (B (W - 1))^2
    float cos_s;             // cos S
    int32_t angle_on;        // S < pi
    float radius;            // support radius R_s (with margin) for culling
    int32_t reach;           // stencil reach in cells
};

struct SceneView {
    const float4* pos;
    const float4* nrm;
    const int32_t* sub_start;
    const int32_t* inv;
    int32_t dims[3];
    float origin[3];
    double h;                // cell edge, as used to bin the points
    int32_t M;
};

// One unit of a flattened (possibly batched) schedule.
struct Chunk {
    int32_t item;   // batch item (0 for single-scene launches)
    int32_t start;  // [start, end) positions within the item's oriented_idx
    int32_t end;
};

struct Item {
    SceneView scene;
    SpinParams p;
    const int32_t* oriented;
    float* images;
    uint32_t* counts;
    int64_t N;
    const int32_t* perm;  // optional iteration -> output position map (learned order)
    // SI_ORDER_SPREAD: loop position w < U spread_full is read from
    // position U ((w / U) spread_mult mod spread_full) + w mod U of perm,
    // U = kSpreadUnit
    int32_t spread_full;  // 0 = off
    int32_t spread_mult;  // coprime to spread_full
};

constexpr int kMaxBases = 64;  // FAC2 batches carried by a launch

struct LaunchDesc {
    Item single;              // the item of a single-scene launch (items == nullptr)
    const Item* items;        // device array for batched launches, else nullptr
    const Chunk* chunks;      // device array, n_chunks
    int32_t n_chunks;
    int32_t dynamic;          // 0: static (see wg_first); 1: atomic claims
    const int32_t* wg_first;  // static only: workgroup k runs chunks
                              // [wg_first[k], wg_first[k+1]); nullptr = chunk k
    const int32_t* n_chunks_dev;  // if set, the chunk count is read from here
    uint32_t* counter;        // 2 words: claim counter, finished workgroups
    int32_t group;            // images per shared candidate pass (1..kMaxGroup)
    int32_t max_w2;           // largest W*W over items (LDS sizing)
    uint32_t ovf_limit;       // in-support count at which an image is redone in 64 bits
    unsigned long long* stat_tested;   // device counters (may be null)
    unsigned long long* stat_support;
    uint32_t* stat_invalid;
    uint32_t* stat_overflow;
    unsigned long long* wg_ns;         // per workgroup busy time (may be null)
    // the device's sticky invalid-index flag (launch_spin fills it in): set
    // to 1 by any launch that meets an oriented index outside [0, M)
    uint32_t* err_flag;
    // emulated heterogeneous workers (si_set_emulated_workers): every
    // emu_every-th workgroup (0 = none) runs 1 + emu_extra times slower,
    // idling (emu_busy 0) or keeping its compute unit busy (emu_busy 1)
    int32_t emu_every;
    float emu_extra;
    int32_t emu_busy;
    int32_t emu_place;           // SI_EMU_EVERY / FIRST / LAST (which workgroups are slow)
    // claims sized by the claiming workgroup (rule = SI_SCHED_WF, AWF or AF;
    // 0 = the chunk table): counter[0] counts claims, counter[2] is the
    // loop's next iteration, each advanced by one atomic addition per claim
    int32_t rule;
    int32_t min_chunk;
    int32_t n_bases;             // FAC2's chunk of each batch (WF, AWF; AF's first chunk)
    int32_t bases[kMaxBases];
    const float* weights;        // WF: one weight per workgroup, summing to the count
    double* adapt;               // AWF: [0] sum of rates, [2] measured workgroups;
                                 // AF: [0] sum of 1/mu, [1] sum of sigma^2/mu, [2] measured
    uint32_t* stat_chunks;       // claims made (may be null)
};

constexpr int kMaxGroup = 8;
constexpr int kBlock = 256;

// Dynamic LDS bytes a launch needs.
size_t spin_lds_bytes(int max_w2, int group);
hipError_t launch_spin(const LaunchDesc& d, int n_wg, hipStream_t s);
// Read and clear the current device's sticky invalid-index flag after the
// work queued on s (synchronises s); *seen = 1 if it was set.
hipError_t take_invalid_flag(hipStream_t s, uint32_t* seen);
int spin_max_wg_per_cu(int max_w2, int group);

// Scene-building kernels.
hipError_t launch_bbox(const float* xyz, int64_t M, float* out6, hipStream_t s);
// key_of[i] = cell * kSubX + x-quarter of point i; counts (n_cells * kSubX)
// are incremented, rank[i] = the point's rank within its key.
hipError_t launch_bin_points(const float* xyz, int64_t M, const Scene& sc, int32_t* key_of,
                             int32_t* rank, int32_t* counts, hipStream_t s);
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, int64_t tmp_n,
                       hipStream_t s);
int64_t scan_tmp_elems(int64_t n);
// 64-bit exclusive scan, out[n] = total; tmp holds scan_tmp_elems(n) values.
hipError_t launch_scan64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s);
hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// perm: iterations sorted by the position of their oriented point in the
// scene's sorted order (cell, then quarter of the cell along x), by a
// counting sort over the M positions; duplicates of one point are in
// arbitrary order.  Temporaries: key, rank (N), counts (M), starts (M + 1),
// tmp (scan_tmp_elems(M)).
hipError_t launch_cell_order(const int32_t* oriented, int64_t N, const Scene& sc, int32_t* key,
                             int32_t* rank, int32_t* counts, int32_t* starts, int32_t* tmp,
                             int32_t* perm, hipStream_t s);
// Same for a batch: iteration t of the concatenated loop belongs to the item
// with item_off[i] <= t < item_off[i+1]; keys are key_base[i] + position, and
// perm[t'] receives the item-local iteration index.  total_keys = sum of the
// items' scene sizes M.
hipError_t launch_cell_order_multi(const Item* items, const int64_t* item_off,
                                   const int64_t* key_base, int n_items, int64_t total_N,
                                   int64_t total_keys, int32_t* key, int32_t* rank,
                                   int32_t* counts, int32_t* starts, int32_t* tmp, int32_t* perm,
                                   hipStream_t s);
hipError_t launch_scatter(const float* xyz, const float* nrm, int64_t M, const int32_t* key_of,
                          const int32_t* rank, const int32_t* sub_start, Scene& sc,
                          hipStream_t s);

// ------------------------------------------------------------ host state --
struct DeviceState {
    bool ready = false;
    int n_cu = 0;
    int wall_khz = 100000;
    int max_lds = 65536;           // bytes of LDS one workgroup may allocate
    uint32_t* counters = nullptr;  // work-counter slots (a static device array), zero between launches
    uint32_t next_slot = 0;
    // chunk-table cache: (kind, N, P, min_chunk, divisor bits) -> device table,
    // uploaded on the stream of its first use (ready: recorded after the
    // copy), with an event per stream recorded after each launch that read
    // it; the least recently used entry is evicted once that stream work is
    // done
    struct Table {
        Chunk* dev = nullptr;
        int n = 0;
        hipEvent_t ready = nullptr;
        std::map<hipStream_t, hipEvent_t> uses;
        uint64_t tick = 0;
        int pins = 0;  // calls between get_table and table_used: never evicted
    };
    std::map<std::tuple<int, int64_t, int, int, uint32_t>, Table> tables;
    uint64_t table_tick = 0;
    // pinned staging of table uploads (one buffer, reused once its last copy is done)
    void* stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t stage_done = nullptr;
    // spin-kernel workgroups per CU: (max W^2, group) -> count
    std::map<std::pair<int, int>, int> wg_per_cu;
};

si_status device_state(DeviceState** out);
// Stream-ordered allocation from the device's memory pool.  The environment
// variable SI_TEST_ALLOC_FAIL, set to a byte count, makes every request of at
// least that many bytes fail with hipErrorOutOfMemory: a test hook for the
// out-of-memory paths.
hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s);
// events registered by si_set_kernel_events on this thread (or null)
void user_kernel_events(hipEvent_t* begin, hipEvent_t* end);
// this thread's si_set_emulated_workers setting, written into a launch
void apply_emulated_workers(LaunchDesc& d);
// this thread's si_set_worker_weights setting (empty = none)
const std::vector<float>& worker_weights();
uint32_t* take_counter(DeviceState* st);
si_status make_params(const si_params* prm, SpinParams* out, double* radius);
si_status check_sched(const si_sched* sc);
SceneView view_of(const Scene& s);
int default_group(int W);
// Stride of SI_ORDER_SPREAD for `full` units: near 0.618 full, coprime to it
// (0 when there is nothing to spread).
int32_t spread_mult(int64_t full);
int fit_group(DeviceState* st, int group, int max_w2);
int auto_workgroups(DeviceState* st, int max_w2, int group);
si_status cell_order(const Scene& sc, const int32_t* oriented, int64_t N, hipStream_t s,
                     int32_t** mem_out, const int32_t** perm_out);
// The chunk table of a schedule on the device, ready for work queued on s
// (uploaded there on first use, or waited for if another stream uploaded it);
// *entry identifies it for table_used, which every successful call must be
// followed by: until then the table is held and cannot be evicted.
si_status get_table(DeviceState* st, int kind, int64_t N, int P, int min_chunk, float divisor,
                    Chunk** out, int* n_out, hipStream_t s, void** entry);
// Release the hold of get_table; with `launched`, first record that work
// queued on s up to now reads the table `entry`.
si_status table_used(DeviceState* st, void* entry, hipStream_t s, bool launched);
si_status run_launch(DeviceState* st, LaunchDesc& d, int n_wg, int max_w2, si_stats* stats,
                     hipStream_t s, int sched_used);
// Learned schedule of one scene, computed on the device in stream order:
// chunk table (its length on the device), iteration -> output permutation,
// all inside `mem` (stream-ordered allocation the caller frees after use).
struct LearnedPlan {
    char* mem = nullptr;
    Chunk* chunks = nullptr;
    int32_t max_chunks = 0;
    const int32_t* n_chunks_dev = nullptr;
    const int32_t* perm = nullptr;
};
// Returns SI_E_UNSUPPORTED when sched->model is NULL.
si_status learned_table(DeviceState* st, const Scene* scene, const int32_t* oriented, int64_t N,
                        const si_params* params, const si_sched* sched, int n_wg, int group,
                        LearnedPlan* plan, hipStream_t s);
si_status features_launch(const Scene& sc, const int32_t* oriented, int64_t N,
                          const si_params* params, float* feats, hipStream_t s);
// Learned schedule of a batched launch (many items), all on the device.
// Buffers in one block laid out by learned_multi_layout (base == nullptr:
// size only).  unit_off (n_items + 1: first unit of each item, kUnit
// iterations per unit) and f11 (n_items: the support-radius feature) are
// filled by the caller; the plan writes perm (total_N: each item's new loop
// order, item-local iterations, at item_off[i]), chunks and *n_chunks.
struct LearnedMulti {
    int64_t* unit_off = nullptr;
    float* f11 = nullptr;
    float* feats = nullptr;
    float* pred = nullptr;
    uint32_t* qcost = nullptr;
    int32_t *ukey = nullptr, *ulen = nullptr, *uitem = nullptr, *urank = nullptr;
    int32_t *hist = nullptr, *ktot = nullptr, *kbase = nullptr, *order = nullptr;
    int64_t *cval = nullptr, *ival = nullptr, *cpre = nullptr, *ipre = nullptr, *ltmp = nullptr;
    int64_t* ends = nullptr;
    int32_t *cut = nullptr, *hcount = nullptr, *hlen = nullptr, *base_len = nullptr;
    int32_t *seg_first = nullptr, *offs = nullptr, *flag = nullptr, *fpre = nullptr;
    int32_t* itmp = nullptr;
    int32_t* perm = nullptr;
    Chunk* chunks = nullptr;
    int32_t* n_chunks = nullptr;
    // summed-volume tables of the items' grids: entry offsets, and the column
    // offsets of the y and z passes, 3 x (n_items + 1) int64; the tables
    int64_t* sat_off = nullptr;
    int32_t* sat = nullptr;
    int64_t sat_pass[3] = {0, 0, 0};  // entries, y columns, z columns
};
int64_t learned_units(const int64_t* item_N, int n_items, int64_t* unit_off_host);
// Host offsets of the items' summed-volume tables: sat_off_host gets
// 3 x (n_items + 1) entries (entries, y columns, z columns); returns the
// total number of table entries.
int64_t sat_offsets(const Item* items, int n_items, int64_t* sat_off_host);
// Whether the features of N images of a grid of these dims come from a
// summed-volume table (built per call) rather than from summing grid rows;
// SI_FEATURES_TABLE = always / never overrides, for tests.
bool use_feature_table(const int32_t* dims, int64_t N);
hipError_t launch_features_multi(const Item* items, const int64_t* item_off, int n_items,
                                 const int32_t* perm_cell, const float* f11,
                                 const int64_t* sat_off, int32_t* sat, const int64_t pass_n[3],
                                 int64_t total_N, float* feats, hipStream_t s);
size_t learned_multi_layout(int n_items, int64_t total_N, int64_t n_units, int P,
                            const int64_t sat_pass[3], LearnedMulti& b, char* base);
hipError_t learned_multi_enqueue(const si_cost_model* model, const LearnedMulti& b,
                                 const Item* items, const int64_t* item_off, int n_items,
                                 const int32_t* perm_cell, int64_t total_N, int64_t n_units, int P,
                                 float divisor, hipStream_t s);
// Largest P the learned schedules accept.
constexpr int kMaxLearnedP = 4096;

// Host chunk tables.
int64_t chunk_sizes(int kind, int64_t N, int P, int min_chunk, float divisor,
                    int64_t* starts, int64_t cap);

}  // namespace si

struct si_scene : si::Scene {};
