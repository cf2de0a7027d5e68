// Spin-image generation kernel for gfx950 (CDNA4).
//
// One persistent launch executes the DOALL loop over images (Section 2.1,
// Algorithm 1).  Each workgroup repeatedly claims a chunk [start, end) of the
// loop (Algorithm 2 is exactly the body run for a claimed chunk): STATIC gives
// workgroup k chunk k; the dynamic techniques of Section 2.2 hand out the
// chunks of a precomputed table through one global atomic counter, which
// replaces the master of the paper's master-worker protocol (Section 3).
//
// Inside a chunk, up to G consecutive images whose grid cells lie close
// together form a group that shares one pass over their common candidate
// points: every candidate point is loaded once (coalesced float4 records of a
// cell-sorted scene) and tested against all G images.  Candidates are the
// points of the grid rows whose cells can hold a point within the support
// radius of some image of the group; rows and their x-extent are culled
// against the support sphere in double precision so that no in-support point
// is ever skipped.
//
// Per pair (beta, alpha as in Algorithm 1):
//   beta = n.(x-p), alpha^2 = |x-p|^2 - beta^2, c = n.n_x
//   bilinear: in = beta <= B W/2  &&  beta > B(1-W/2)  &&  alpha^2 < (B(W-1))^2  [&& c >= cos S]
//   ceil:     in = beta <  B(W/2+1) && beta >= B(1-W/2) && alpha^2 <= (B(W-1))^2 [&& c >= cos S]
// which are the extent conditions 0 <= v < W-1, u < W-1 (bilinear) and
// 0 <= ceil(v), ceil(u) < W (ceil) of v = W/2 - beta/B, u = alpha/B written in
// scene units.  Images accumulate in LDS as unsigned 16.16 fixed point with
// integer atomics: each in-support pair adds exactly 65536 (its four bilinear
// weights are rounded so that they sum to 65536), so an image is a sum of
// integers and does not depend on the order in which pairs arrive.  An image
// whose in-support count reaches 65536 could wrap a 32-bit bin; it is redone
// with 64-bit LDS accumulators.
#include "si_internal.h"
#include "adaptive.h"

#include <map>
#include <mutex>

namespace si {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kInfo = 64;     // images whose descriptors are staged at once
static_assert(kInfo == 64, "group formation reads staged image l from lane l of a wave");
constexpr int kMaxRows = 64;  // candidate rows per group (one lane each)

struct __attribute__((aligned(16))) ImgInfo {
    float px, py, pz;
    int32_t out;      // output position, -1 = invalid index
    float nx, ny, nz;
    int32_t cell;     // linear cell id, -1 = invalid index
    int32_t cx, cy, cz, pad;  // cell coordinates
};

__device__ __forceinline__ float rfl(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double rfl(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = (uint32_t)rfl((int)(uint32_t)b), hi = (uint32_t)rfl((int)(uint32_t)(b >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}
template <typename T>
__device__ __forceinline__ T* rfl(T* v) {
    const uint64_t b = (uint64_t)v;
    const uint64_t lo = (uint32_t)rfl((int)(uint32_t)b), hi = (uint32_t)rfl((int)(uint32_t)(b >> 32));
    return (T*)((hi << 32) | lo);
}

// Per-item values the whole workgroup shares, pinned to scalar registers so
// that comparisons against them and branches on them stay wave-uniform.
__device__ __forceinline__ SpinParams uniform(const SpinParams& a) {
    SpinParams b;
    b.W = rfl(a.W);
    b.mode = rfl(a.mode);
    b.half = rfl(a.half);
    b.inv_bin = rfl(a.inv_bin);
    b.beta_lo = rfl(a.beta_lo);
    b.beta_hi = rfl(a.beta_hi);
    b.alpha2_max = rfl(a.alpha2_max);
    b.cos_s = rfl(a.cos_s);
    b.angle_on = rfl(a.angle_on);
    b.radius = rfl(a.radius);
    b.reach = rfl(a.reach);
    return b;
}
__device__ __forceinline__ SceneView uniform(const SceneView& a) {
    SceneView b;
    b.pos = rfl(a.pos);
    b.nrm = rfl(a.nrm);
    b.sub_start = rfl(a.sub_start);
    b.inv = rfl(a.inv);
    for (int k = 0; k < 3; ++k) {
        b.dims[k] = rfl(a.dims[k]);
        b.origin[k] = rfl(a.origin[k]);
    }
    b.h = rfl(a.h);
    b.M = rfl(a.M);
    return b;
}

__device__ __forceinline__ void cell_xyz(int cell, const int* dims, int& cx, int& cy, int& cz) {
    cx = cell % dims[0];
    int t = cell / dims[0];
    cy = t % dims[1];
    cz = t / dims[1];
}

// Position of an in-support pair in the image, given beta and alpha^2.
// Bilinear: 16.16 fixed-point V = round(v 2^16), U = round(u 2^16) of
// v = W/2 - beta/B, u = alpha/B, kept below (W - 1) 2^16 so that the 2 x 2
// footprint stays inside; they tolerate the 1-ulp hardware square root (a
// one-ulp change of u moves at most one quantisation step).  alpha^2 of an
// in-support pair is finite, so the clamp at zero is a median.
__device__ __forceinline__ void bilinear_pos(const SpinParams& p, float beta, float a2,
                                             uint32_t& V, uint32_t& U) {
    const float s = 65536.0f;
    const float top = (float)(((p.W - 1) << 16) - 1);
    a2 = __builtin_amdgcn_fmed3f(a2, 0.0f, 3.0e38f);
    const float vf = fmaf(-beta, p.inv_bin * s, fmaf(p.half, s, 0.5f));
    const float uf = fmaf(__builtin_amdgcn_sqrtf(a2), p.inv_bin * s, 0.5f);
    V = (uint32_t)__builtin_amdgcn_fmed3f(vf, 0.0f, top);
    U = (uint32_t)__builtin_amdgcn_fmed3f(uf, 0.0f, top);
}
// The four weights of (V, U), rounded so that they sum to exactly 65536:
// w00 at (row, col), w01 at (row, col + 1), w10 at (row + 1, col), w11 at
// (row + 1, col + 1) with row = V >> 16, col = U >> 16.
__device__ __forceinline__ void bilinear_weights(uint32_t V, uint32_t U, uint32_t& w00,
                                                 uint32_t& w01, uint32_t& w10, uint32_t& w11) {
    const uint32_t qa = V & 0xffffu, qb = U & 0xffffu;
    w11 = (__umul24(qa, qb) + 32768u) >> 16;
    w10 = qa - w11;
    w01 = qb - w11;
    w00 = 65536u - qb - w10;
}
// Ceil: bin (k, l) = (ceil v, ceil u) clamped to the image, with the
// correctly rounded square root since ceil(alpha/B) jumps at integers.
__device__ __forceinline__ void ceil_pos(const SpinParams& p, float beta, float a2, int& k, int& l) {
    a2 = __builtin_amdgcn_fmed3f(a2, 0.0f, 3.0e38f);
    const float v = fmaf(-beta, p.inv_bin, p.half);
    const float u = sqrtf(a2) * p.inv_bin;
    k = min(max((int)ceilf(v), 0), p.W - 1);
    l = min(max((int)ceilf(u), 0), p.W - 1);
}

// Accumulate one in-support pair into a u32 or u64 LDS image.  Every path
// that bins a pair computes its position and weights with the functions
// above, so results do not depend on which path ran.
template <int MODE, typename Acc>
__device__ __forceinline__ void bin_pair(Acc* img, const SpinParams& p, float beta, float a2) {
    const int W = p.W;
    if (MODE == SI_BIN_BILINEAR) {
        uint32_t V, U, w00, w01, w10, w11;
        bilinear_pos(p, beta, a2, V, U);
        bilinear_weights(V, U, w00, w01, w10, w11);
        Acc* r0 = img + __umul24(V >> 16, (uint32_t)W) + (U >> 16);
        atomicAdd(r0, (Acc)w00);
        atomicAdd(r0 + 1, (Acc)w01);
        atomicAdd(r0 + W, (Acc)w10);
        atomicAdd(r0 + W + 1, (Acc)w11);
    } else {
        int k, l;
        ceil_pos(p, beta, a2, k, l);
        atomicAdd(img + k * W + l, (Acc)65536u);
    }
}

struct GroupImg {
    float px, py, pz, nx, ny, nz;
};

// Test every candidate of the group's rows against `ng` images.
// acc: ng images of W*W accumulators.  cnt: per-thread in-support counts.
template <int MODE, int G, typename Acc>
__device__ __forceinline__ void candidate_pass(const SceneView& sc, const SpinParams& p,
                                               const GroupImg* gi, int ng, Acc* acc,
                                               const int* row_start, const int* row_pref,
                                               int n_rows, uint32_t* cnt) {
    const int W = p.W;
    const int w2 = W * W;
    const int total = row_pref[n_rows];
    int r = 0;
    for (int k = threadIdx.x; k < total; k += kBlock) {
        while (row_pref[r + 1] <= k) ++r;
        const int j = row_start[r] + (k - row_pref[r]);
        const float4 x = sc.pos[j];
        const float4 m = sc.nrm[j];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (g < ng) {
                const float dx = x.x - gi[g].px;
                const float dy = x.y - gi[g].py;
                const float dz = x.z - gi[g].pz;
                const float beta = fmaf(gi[g].nz, dz, fmaf(gi[g].ny, dy, gi[g].nx * dx));
                const float dd = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                const float a2 = fmaf(-beta, beta, dd);
                bool in;
                if (MODE == SI_BIN_BILINEAR)
                    in = (beta <= p.beta_hi) & (beta > p.beta_lo) & (a2 < p.alpha2_max);
                else
                    in = (beta < p.beta_hi) & (beta >= p.beta_lo) & (a2 <= p.alpha2_max);
                if (p.angle_on) {
                    const float c = fmaf(gi[g].nz, m.z, fmaf(gi[g].ny, m.y, gi[g].nx * m.x));
                    in = in & (c >= p.cos_s);
                }
                if (in) {
                    bin_pair<MODE>(acc + g * w2, p, beta, a2);
                    cnt[g] += 1;
                }
            }
        }
    }
}

// Queue of one wave's in-support pairs, three arrays of kQueue words: beta,
// alpha^2 and the LDS byte address of the image's accumulators, so that one
// address serves an entry's three words.
constexpr int kQueue = 224;  // entries per wave
constexpr int kRounds = (kQueue + 63) / 64;  // binning rounds of a full queue
struct WaveQueue {
    float beta[kQueue];
    float a2[kQueue];
    uint32_t img[kQueue];
};

typedef __attribute__((address_space(1))) const f32x4 gf32x4;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

__device__ __forceinline__ uint32_t lds_address(const void* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}
__device__ __forceinline__ uint32_t* lds_pointer(uint32_t a) {
    return (uint32_t*)(lds_u32*)(uintptr_t)a;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Bin the queued pairs of this wave densely: lane l takes entries l*T ..
// l*T+T-1 (T = rounds), so entries appended together (neighbouring points,
// often the same bins) go to different rounds.
template <int MODE>
__device__ __forceinline__ void flush_queue(const SpinParams& p, const WaveQueue* q, int qn) {
    const int lane = threadIdx.x & 63;
    const uint32_t row_bytes = (uint32_t)p.W * 4u;
    wave_sync_lds();
    // every round's entry is read before any is binned (indices clamped to
    // the queue; entries at or beyond qn are read but not binned)
    const int T = (qn + 63) >> 6;
    float bq[kRounds], aq[kRounds];
    uint32_t iq[kRounds];
#pragma unroll
    for (int t = 0; t < kRounds; ++t) {
        const int e = min(lane * T + t, kQueue - 1);
        bq[t] = q->beta[e];
        aq[t] = q->a2[e];
        iq[t] = q->img[e];
    }
#pragma unroll
    for (int t = 0; t < kRounds; ++t) {
        const int e = lane * T + t;
        if (t < T && e < qn) {
            const float beta = bq[t], a2 = aq[t];
            const uint32_t img = iq[t];
            if (MODE == SI_BIN_BILINEAR) {
                uint32_t V, U, w00, w01, w10, w11;
                bilinear_pos(p, beta, a2, V, U);
                bilinear_weights(V, U, w00, w01, w10, w11);
                uint32_t* r0 = lds_pointer(img + __umul24(V >> 16, row_bytes) + ((U >> 16) << 2));
                atomicAdd(r0, w00);
                atomicAdd(r0 + 1, w01);
                uint32_t* r1 = lds_pointer(img + __umul24(V >> 16, row_bytes) + row_bytes + ((U >> 16) << 2));
                atomicAdd(r1, w10);
                atomicAdd(r1 + 1, w11);
            } else {
                int k, l;
                ceil_pos(p, beta, a2, k, l);
                atomicAdd(lds_pointer(img + (uint32_t)(k * p.W + l) * 4u), 65536u);
            }
        }
    }
    wave_sync_lds();
}

// Test every candidate of the group's rows against `ng` images; pairs in
// support are appended to the wave's LDS queue and binned when it fills.
// Each wave takes a contiguous quarter of the candidate list (a multiple of
// 64) and walks it 64 at a time, the next candidates' loads issued before the
// current ones are tested.  The loop bounds and the queue fill are
// wave-uniform, so loop control stays scalar.
// cnt: per-image in-support counts of this wave (wave-uniform).
template <int MODE, int G, bool ANGLE>
__device__ __forceinline__ void candidate_pass_q(const SceneView& sc, const SpinParams& p,
                                                 const GroupImg* gi, int ng, uint32_t* acc,
                                                 const int* row_start, const int* row_pref,
                                                 int n_rows, WaveQueue* q, uint32_t* cnt) {
    const int lane = threadIdx.x & 63;
    const int wave = rfl((int)(threadIdx.x >> 6));
    const int total = rfl(row_pref[n_rows]);
    // the wave's queue at a scalar LDS address, so that appends compute one
    // vector address per lane
    q = (WaveQueue*)lds_pointer((uint32_t)rfl((int)lds_address(q)));
    const char* gpos = (const char*)sc.pos;
    const char* gnrm = (const char*)sc.nrm;
    const int w2p = p.W * p.W + 4;  // padded image stride
    uint32_t img_at[G];
#pragma unroll
    for (int g = 0; g < G; ++g) img_at[g] = lds_address(acc + g * w2p);
    const int quarter = ((total + kBlock - 1) / kBlock) * 64;
    const int w_beg = min(total, wave * quarter), w_end = min(total, w_beg + quarter);
    // row cursor: the lane's current row ends at candidate r_hi, and its
    // candidate k is point k + r_off; first row: the last r with
    // row_pref[r] <= this lane's first k
    int r = 0;
    {
        const int k0 = min(w_beg + lane, max(total - 1, 0));
        int hi = max(n_rows - 1, 0);
        while (r < hi) {
            const int mid = (r + hi + 1) >> 1;
            if (row_pref[mid] <= k0) r = mid; else hi = mid - 1;
        }
    }
    int r_hi = row_pref[r + 1], r_off = row_start[r] - row_pref[r];
    auto fetch = [&](int k, f32x4& x, f32x4& m) {
        while (k >= r_hi) {
            ++r;
            r_off = row_start[r] - r_hi;
            r_hi = row_pref[r + 1];
        }
        const uint32_t off = (uint32_t)(k + r_off) << 4;
        x = *(gf32x4*)(gpos + off);
        m = *(gf32x4*)(gnrm + off);
    };
    int qn = 0;
    f32x4 xn = {0.0f, 0.0f, 0.0f, 0.0f}, mn = xn;
    int kb = w_beg;
    if (lane < w_end - kb) fetch(kb + lane, xn, mn);
    for (; kb < w_end; kb += 64) {
        const f32x4 x = xn, m = mn;
        const int lim = w_end - kb;
        const bool valid = lane < lim;
        const uint64_t vmask = __builtin_amdgcn_ballot_w64(valid);
        if (lane < lim - 64) fetch(kb + 64 + lane, xn, mn);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (g < ng) {
                const float dx = x[0] - gi[g].px;
                const float dy = x[1] - gi[g].py;
                const float dz = x[2] - gi[g].pz;
                const float beta = fmaf(gi[g].nz, dz, fmaf(gi[g].ny, dy, gi[g].nx * dx));
                const float dd = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                const float a2 = fmaf(-beta, beta, dd);
                // one ballot per comparison: each is that compare's lane mask
                bool b0, b1, b2;
                if (MODE == SI_BIN_BILINEAR) {
                    b0 = beta <= p.beta_hi; b1 = beta > p.beta_lo; b2 = a2 < p.alpha2_max;
                } else {
                    b0 = beta < p.beta_hi; b1 = beta >= p.beta_lo; b2 = a2 <= p.alpha2_max;
                }
                uint64_t mask = __builtin_amdgcn_ballot_w64(b0) & __builtin_amdgcn_ballot_w64(b1) &
                                __builtin_amdgcn_ballot_w64(b2) & vmask;
                bool in = b0 & b1 & b2 & valid;
                if (ANGLE) {
                    const float c = fmaf(gi[g].nz, m[2], fmaf(gi[g].ny, m[1], gi[g].nx * m[0]));
                    const bool b3 = c >= p.cos_s;
                    mask &= __builtin_amdgcn_ballot_w64(b3);
                    in = in & b3;
                }
                if (mask) {
                    if (in) {
                        // rank among the passing lanes; the queue's fill is
                        // added to the scalar base
                        const uint32_t slot = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                        (q->beta + qn)[slot] = beta;
                        (q->a2 + qn)[slot] = a2;
                        (q->img + qn)[slot] = img_at[g];
                    }
                    const int c = __popcll(mask);
                    qn += c;
                    cnt[g] += c;
                    if (__builtin_expect(qn > kQueue - 64, 0)) {
                        flush_queue<MODE>(p, q, qn);
                        qn = 0;
                    }
                }
            }
        }
    }
    if (qn) flush_queue<MODE>(p, q, qn);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Rows (z, y) of grid cells that may hold candidates of the group, each with
// the contiguous run of points, in quarter-cell steps along x (the sort key
// of the scene), that meets the support sphere and the beta slab of some
// image of the group (float32 relative to the image's point; the sphere, the
// slab and the x range are widened by a margin of 2e-6 of the scene's largest
// coordinate, many ulp of it, so rounding never cuts a candidate).  Two
// phases, both called by every thread of the block: rows_cull: thread t
// bounds row t % 64 against images t / 64 and t / 64 + 4 into the key range
// part_x0/part_x1[t]; rows_emit (after a barrier): lane r of wave 0 merges
// the four partial ranges of row r, looks them up in sub_start and writes
// row_start / row_pref (exclusive prefix of run lengths) / n_rows.
__device__ __forceinline__ void rows_cull(const SceneView& sc, const SpinParams& p,
                                          const GroupImg* gi, const int* gcx, int ng,
                                          const int lo[3], const int hi[3], int* part_x0,
                                          int* part_x1) {
    const int t = threadIdx.x;
    const int r = t & 63, q = rfl(t >> 6);
    const int ny_rows = hi[1] - lo[1] + 1;
    const int nz_rows = hi[2] - lo[2] + 1;
    const int n_rows = ny_rows * nz_rows;  // <= kMaxRows by construction
    int x0 = 0x7fffffff, x1 = -1;
    if (r < n_rows) {
        const int cy = lo[1] + r % ny_rows;
        const int cz = lo[2] + r / ny_rows;
        // eps: 2e-6 of the largest coordinate, against row bounds and point
        // offsets that are each a few ulp of it off the exact ones; the
        // chord's sqrt near zero cancellation is covered since eps R > ulp(R^2)
        // for every cell size h >= R / 4
        const float h = (float)sc.h;
        const float qx = (float)kSubX / h;
        float mag = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            mag = fmaxf(mag, fabsf(sc.origin[a]) + (float)sc.dims[a] * h);
        const float eps = 2e-6f * mag + 1e-6f;
        const float R = p.radius + eps;
        const float R2 = R * R;
        // float32 beta is accurate to ~1e-6; the slab keeps a much wider margin
        const float slab_eps = 1e-4f * fmaxf(1.0f, p.radius) + eps;
#pragma unroll
        for (int g = 0; g < kMaxGroup; ++g) {
            if (g >= ng) break;
            if ((g & 3) != q) continue;  // wave q takes images q and q + 4
            const float py = gi[g].py, pz = gi[g].pz, px = gi[g].px;
            if (!(py == py) || !(pz == pz) || !(px == px)) continue;  // invalid image
            // the row's y-z box relative to p
            const float ylo = (sc.origin[1] - py) + (float)cy * h, yhi = ylo + h;
            const float zlo = (sc.origin[2] - pz) + (float)cz * h, zhi = zlo + h;
            const float dy = fmaxf(0.0f, fmaxf(ylo, -yhi));
            const float dz = fmaxf(0.0f, fmaxf(zlo, -zhi));
            const float d2 = fmaf(dz, dz, dy * dy);
            if (d2 > R2) continue;
            const float half_chord = sqrtf(R2 - d2);
            float xa = -half_chord, xb = half_chord;
            // slab beta_lo < n.(x - p) <= beta_hi over the row's y-z box
            const float nx = gi[g].nx, ny = gi[g].ny, nz = gi[g].nz;
            const float ty0 = ny * ylo, ty1 = ny * yhi;
            const float tz0 = nz * zlo, tz1 = nz * zhi;
            const float tmin = fminf(ty0, ty1) + fminf(tz0, tz1);
            const float tmax = fmaxf(ty0, ty1) + fmaxf(tz0, tz1);
            const float A = p.beta_lo - slab_eps - tmax;  // bound of nx (x - px)
            const float Bv = p.beta_hi + slab_eps - tmin;
            if (fabsf(nx) > 1e-20f) {
                const float inv_nx = __builtin_amdgcn_rcpf(nx);
                float s0 = A * inv_nx, s1 = Bv * inv_nx;
                if (s0 > s1) { const float tt = s0; s0 = s1; s1 = tt; }
                xa = fmaxf(xa, s0 - fabsf(s0) * 1e-6f - eps);
                xb = fminf(xb, s1 + fabsf(s1) * 1e-6f + eps);
            } else if (A > 0.0f || Bv < 0.0f) {
                continue;
            }
            if (!(xa <= xb)) continue;
            // keys along the row: kSubX per cell
            const float ox = px - sc.origin[0];
            const float fa = floorf((ox + xa - eps) * qx);
            const float fb = floorf((ox + xb + eps) * qx);
            const int a = (int)fmaxf(-1.0f, fminf(fa, 1.0e9f));
            const int b = (int)fmaxf(-1.0f, fminf(fb, 1.0e9f));
            if (p.reach == 0) {
                // single-cell scene: the paper's loop over all M points
                x0 = 0;
                x1 = kSubX - 1;
                continue;
            }
            x0 = min(x0, max(a, (gcx[g] - p.reach) * kSubX));
            x1 = max(x1, min(b, (gcx[g] + p.reach) * kSubX + kSubX - 1));
        }
        // this thread's part of the row's run, as point indices
        x0 = max(x0, 0);
        x1 = min(x1, sc.dims[0] * kSubX - 1);
        if (x1 >= x0) {
            const int base = (cz * sc.dims[1] + cy) * sc.dims[0] * kSubX;
            const int st = sc.sub_start[base + x0];
            x1 = sc.sub_start[base + x1 + 1];
            x0 = st;
        } else {
            x0 = 0x7fffffff;
            x1 = -1;
        }
    }
    part_x0[t] = x0;
    part_x1[t] = x1;
}

__device__ __forceinline__ void rows_emit(const SceneView& sc, const int lo[3], const int hi[3],
                                          bool any_valid, const int* part_x0,
                                          const int* part_x1, int* row_start, int* row_pref,
                                          int* n_rows_out) {
    const int lane = threadIdx.x;  // caller guarantees threadIdx.x < 64
    const int ny_rows = any_valid ? hi[1] - lo[1] + 1 : 0;
    const int nz_rows = any_valid ? hi[2] - lo[2] + 1 : 0;
    const int n_rows = ny_rows * nz_rows;
    int len = 0, start = 0;
    if (lane < n_rows) {
        // the partial runs are key ranges of one row, so the point range of
        // their span is [min of starts, max of ends)
        int x0 = part_x0[lane], x1 = part_x1[lane];
#pragma unroll
        for (int q = 1; q < kBlock / 64; ++q) {
            x0 = min(x0, part_x0[lane + 64 * q]);
            x1 = max(x1, part_x1[lane + 64 * q]);
        }
        if (x1 > x0) {
            start = x0;
            len = x1 - x0;
        }
    }
    // inclusive scan of len over the wave
    int incl = len;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane < n_rows) {
        row_start[lane] = start;
        row_pref[lane + 1] = incl;
    }
    if (lane == 0) {
        row_pref[0] = 0;
        *n_rows_out = n_rows;
    }
}

template <int G>
__device__ __forceinline__ void run_group_pass(const SceneView& sc, const SpinParams& p,
                                               const GroupImg* gi, int ng, uint32_t* acc,
                                               const int* row_start, const int* row_pref,
                                               int n_rows, WaveQueue* q, uint32_t* cnt) {
    if (p.mode == SI_BIN_BILINEAR) {
        if (p.angle_on)
            candidate_pass_q<SI_BIN_BILINEAR, G, true>(sc, p, gi, ng, acc, row_start, row_pref,
                                                       n_rows, q, cnt);
        else
            candidate_pass_q<SI_BIN_BILINEAR, G, false>(sc, p, gi, ng, acc, row_start, row_pref,
                                                        n_rows, q, cnt);
    } else {
        if (p.angle_on)
            candidate_pass_q<SI_BIN_CEIL, G, true>(sc, p, gi, ng, acc, row_start, row_pref,
                                                   n_rows, q, cnt);
        else
            candidate_pass_q<SI_BIN_CEIL, G, false>(sc, p, gi, ng, acc, row_start, row_pref,
                                                    n_rows, q, cnt);
    }
}

}  // namespace

// EMU: the build that can emulate slower workers (si_set_emulated_workers);
// the default build has none of that code.
template <bool EMU>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) k_spin(LaunchDesc d) {
    extern __shared__ uint4 acc_lds[];
    uint32_t* acc = reinterpret_cast<uint32_t*>(acc_lds);
    __shared__ ImgInfo s_info[kInfo];
    __shared__ int s_row_start[kMaxRows];
    __shared__ int s_row_pref[kMaxRows + 1];
    __shared__ int s_n_rows;
    __shared__ uint32_t s_cnt[kMaxGroup];
    __shared__ int s_step;
    __shared__ int s_cs, s_ce;                   // EMU, worker-sized claims: the chunk
    __shared__ unsigned long long s_until;       // EMU: end of an emulated slowdown
    __shared__ int s_slow;                       // EMU: this workgroup is an emulated slow one
    // EMU build, used by thread 0 only: when the current chunk and group
    // began, the workgroup's measurements for AWF (sums over its chunks k of
    // k n_k and k t_k, its rate) and AF (Welford sums of per-image times, and
    // what it last added to the launch-wide sums), and its claims
    __shared__ struct {
        unsigned long long t_chunk, t_group;
        double aw_a, aw_b, aw_rate;
        double af_n, af_mean, af_m2, af_c1, af_c2;
        int aw_k, af_meas;
        uint32_t claims;
        int first_claim;
    } s_m;
    __shared__ WaveQueue s_q[kBlock / 64];
    // the row culling's partial runs live in the queues, which are empty
    // between candidate passes (barriers separate the two uses)
    int* s_part_x0 = reinterpret_cast<int*>(&s_q[0]);
    int* s_part_x1 = s_part_x0 + kBlock;

    const int tid = threadIdx.x;
    const uint64_t t_begin = wall_clock64();
    const int n_chunks = d.n_chunks_dev ? rfl(*d.n_chunks_dev) : d.n_chunks;
    unsigned long long my_tested = 0, my_support = 0;
    uint32_t my_invalid = 0, my_overflow = 0;
    int local = 0;  // static: chunks this workgroup has taken
    if (EMU && tid == 0) {
        memset(&s_m, 0, sizeof(s_m));
        s_slow = d.emu_every > 0 && d.emu_place == SI_EMU_EVERY &&
                 blockIdx.x % (unsigned)d.emu_every == 0;
    }

    for (;;) {
        if (tid == 0) {
            int step;
            if (EMU && d.rule) {
                // claim sized by this workgroup (WF / AWF / AF): take a claim
                // index (its batch, for WF and AWF), size the chunk, then
                // advance the loop's next iteration by that size; a start at
                // or past the end means the loop is done (no retries: every
                // workgroup makes progress with two atomic additions)
                uint32_t* next_it = d.counter + 2;
                const int64_t N = d.single.N;
                const int P = (int)gridDim.x;
                const int64_t mc = d.min_chunk;
                const uint32_t r = atomicAdd(d.counter, 1u);
                const int64_t b = (int64_t)(r / (uint32_t)P);
                const int64_t base = b < d.n_bases ? d.bases[b] : mc;
                const int64_t nxt = (int64_t)__hip_atomic_load(next_it, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                const int64_t R = N - nxt;
                int64_t k = 0;
                if (R > 0) {
                    if (d.rule == SI_SCHED_WF) {
                        k = wf_chunk((double)d.weights[blockIdx.x], base, R, mc);
                    } else {
                        const double s0 = __hip_atomic_load(&d.adapt[0], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                        const double s1 = __hip_atomic_load(&d.adapt[1], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                        const int nm = (int)__hip_atomic_load(&d.adapt[2], __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
                        if (d.rule == SI_SCHED_AWF) {
                            k = wf_chunk(awf_weight(s_m.aw_rate, s0, nm, P), base, R, mc);
                        } else if (s_m.af_meas && nm > 0 && s0 > 0.0) {
                            double D, T;
                            af_terms(s1, s0, nm, P, &D, &T);
                            k = af_chunk(D, T, R, s_m.af_mean, mc);
                        } else {
                            k = clamp_chunk((double)d.bases[0], R, mc);
                        }
                    }
                }
                // R was read before the addition: the chunk is clamped to the end
                const int64_t cs = k > 0 ? (int64_t)atomicAdd(next_it, (uint32_t)k) : N;
                const int64_t ce = cs < N ? (cs + k < N ? cs + k : N) : N;
                s_cs = (int)(cs < N ? cs : N);
                s_ce = (int)ce;
                step = cs < N ? 0 : n_chunks;
                if (cs < N && s_m.claims++ == 0) s_m.first_claim = (int)r;
            } else if (d.dynamic) {
                step = (int)atomicAdd(d.counter, 1u);
            } else if (d.wg_first) {
                step = d.wg_first[blockIdx.x] + local;
                if (step >= d.wg_first[blockIdx.x + 1]) step = n_chunks;
            } else {
                step = local == 0 ? (int)blockIdx.x : n_chunks;
            }
            s_step = step;
            if (EMU) {
                s_m.t_chunk = s_m.t_group = wall_clock64();
                if (local == 0 && d.emu_every > 0 && d.emu_place != SI_EMU_EVERY) {
                    // slow by the place of this workgroup's first claim among
                    // all claims (STATIC: its index); a workgroup that finds
                    // the loop done claims nothing
                    const int first = d.rule ? (int)(s_m.claims ? s_m.first_claim : 0x7fffffff)
                                             : step;
                    const int n_slow = (int)gridDim.x / d.emu_every;
                    s_slow = d.emu_place == SI_EMU_FIRST ? first < n_slow
                                                         : first >= (int)gridDim.x - n_slow;
                }
            }
        }
        ++local;
        __syncthreads();
        const int step = rfl(s_step);
        if (step >= n_chunks) break;
        Chunk ch;
        if (EMU && d.rule) {
            ch.item = 0;
            ch.start = s_cs;
            ch.end = s_ce;
        } else {
            ch = d.chunks[step];
        }
        const int item_id = rfl(ch.item);
        const int c_start = rfl(ch.start);
        const int c_end = rfl(ch.end);
        const Item& it = d.items ? d.items[item_id] : d.single;
        const SceneView sc = uniform(it.scene);
        const SpinParams p = uniform(it.p);
        const int W = p.W;
        const int w2 = W * W;
        // images per group: keep the LDS footprint of the launch (group x
        // max_w2); items of a smaller W take more images, at most
        // max(group, 4) (the 8-image pass spills scalar registers, which
        // pays only for W <= 16 images, whose groups have few candidates
        // and whose per-group work dominates: those take up to 8)
        const int G_item = min(w2 <= 256 ? kMaxGroup : max(d.group, 4),
                               min(kMaxGroup, max(1, (d.group * (d.max_w2 + 4)) / (w2 + 4))));
        // cells a group may span per axis beyond the first, and rows available
        const int span_lim = max(0, min(1, 7 - 2 * p.reach));

        for (int b0 = c_start; b0 < c_end; b0 += kInfo) {
            const int nb = min(kInfo, c_end - b0);
            __syncthreads();  // s_info reuse
            if (tid < nb) {
                int w = b0 + tid;
                if (it.spread_full > 1 && w < it.spread_full * kSpreadUnit)
                    w = (int)(((long long)(w / kSpreadUnit) * it.spread_mult) % it.spread_full) *
                            kSpreadUnit +
                        (w & (kSpreadUnit - 1));
                const int out = it.perm ? it.perm[w] : w;
                const int o = it.oriented[out];
                ImgInfo inf;
                if (o >= 0 && o < sc.M) {
                    const int sp = sc.inv[o];
                    const float4 a = sc.pos[sp];
                    const float4 n = sc.nrm[sp];
                    inf.px = a.x; inf.py = a.y; inf.pz = a.z;
                    inf.nx = n.x; inf.ny = n.y; inf.nz = n.z;
                    inf.cell = __float_as_int(a.w);
                    cell_xyz(inf.cell, sc.dims, inf.cx, inf.cy, inf.cz);
                    inf.out = out;
                } else {
                    const float qnan = __int_as_float(0x7fc00000);
                    inf.px = inf.py = inf.pz = qnan;
                    inf.nx = inf.ny = inf.nz = qnan;
                    inf.cell = -1;
                    inf.cx = inf.cy = inf.cz = 0;
                    inf.out = -1 - out;  // invalid: encode the output position
                }
                s_info[tid] = inf;
            }
            __syncthreads();

            int cur = 0;
            while (cur < nb) {
                // ---- form a group (every wave computes the same answer) ----
                // lane l of each wave holds staged image l (kInfo = 64 lanes);
                // the serial scan below reads it with readlane, so its
                // decisions are scalar and wait on no LDS round trip
                const int l = tid & 63;
                const ImgInfo li = s_info[l < nb ? l : 0];
                int lo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff};
                int hi[3] = {-1, -1, -1};
                int ng = 0;
                while (ng < G_item && cur + ng < nb) {
                    const int i = cur + ng;
                    if (__builtin_amdgcn_readlane(li.cell, i) >= 0) {
                        const int c[3] = {__builtin_amdgcn_readlane(li.cx, i),
                                          __builtin_amdgcn_readlane(li.cy, i),
                                          __builtin_amdgcn_readlane(li.cz, i)};
                        int nlo[3], nhi[3];
                        bool ok = true;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            nlo[a] = min(lo[a], c[a]);
                            nhi[a] = max(hi[a], c[a]);
                            if (nhi[a] - nlo[a] > span_lim) ok = false;
                        }
                        if (!ok && ng > 0) break;
#pragma unroll
                        for (int a = 0; a < 3; ++a) { lo[a] = nlo[a]; hi[a] = nhi[a]; }
                    }
                    ++ng;
                }
                int gcx[kMaxGroup];
                GroupImg gi[kMaxGroup];
#pragma unroll
                for (int g = 0; g < kMaxGroup; ++g) {
                    if (g >= ng) break;
                    const int i = cur + g;
                    gcx[g] = __builtin_amdgcn_readlane(li.cx, i);
                    gi[g].px = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(li.px), i));
                    gi[g].py = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(li.py), i));
                    gi[g].pz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(li.pz), i));
                    gi[g].nx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(li.nx), i));
                    gi[g].ny = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(li.ny), i));
                    gi[g].nz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(li.nz), i));
                }
                const bool any_valid = hi[0] >= 0;
                int rlo[3], rhi[3];
                for (int a = 0; a < 3; ++a) {
                    rlo[a] = any_valid ? max(lo[a] - p.reach, 0) : 0;
                    rhi[a] = any_valid ? min(hi[a] + p.reach, sc.dims[a] - 1) : -1;
                }

                // ---- zero accumulators + counts; cull the rows (all waves) ----
                {
                    uint4* a4 = reinterpret_cast<uint4*>(acc);
                    const int n4 = (ng * (w2 + 4) + 3) / 4;
                    for (int i = tid; i < n4; i += kBlock) a4[i] = make_uint4(0, 0, 0, 0);
                    if (tid < kMaxGroup) s_cnt[tid] = 0;
                }
                rows_cull(sc, p, gi, gcx, ng, rlo, rhi, s_part_x0, s_part_x1);
                __syncthreads();
                if (tid < 64)
                    rows_emit(sc, rlo, rhi, any_valid, s_part_x0, s_part_x1, s_row_start,
                              s_row_pref, &s_n_rows);
                __syncthreads();
                const int n_rows = rfl(s_n_rows);

                // ---- candidate pass ----
                uint32_t cnt[kMaxGroup];
#pragma unroll
                for (int g = 0; g < kMaxGroup; ++g) cnt[g] = 0;
                WaveQueue* q = &s_q[tid >> 6];
                if (ng > 4)
                    run_group_pass<8>(sc, p, gi, ng, acc, s_row_start, s_row_pref, n_rows, q,
                                      cnt);
                else if (ng > 2)
                    run_group_pass<4>(sc, p, gi, ng, acc, s_row_start, s_row_pref, n_rows, q,
                                      cnt);
                else if (ng > 1)
                    run_group_pass<2>(sc, p, gi, ng, acc, s_row_start, s_row_pref, n_rows, q,
                                      cnt);
                else
                    run_group_pass<1>(sc, p, gi, ng, acc, s_row_start, s_row_pref, n_rows, q,
                                      cnt);
#pragma unroll
                for (int g = 0; g < kMaxGroup; ++g) {
                    if (g < ng && (tid & 63) == 0 && cnt[g]) atomicAdd(&s_cnt[g], cnt[g]);
                }
                if (tid == 0) my_tested += (unsigned long long)s_row_pref[n_rows] * ng;
                __syncthreads();

                // ---- write the group's images and counts ----
                int redo_mask = 0;
                for (int g = 0; g < ng; ++g) {
                    const int out_code = s_info[cur + g].out;
                    const uint32_t c = s_cnt[g];
                    const bool valid = out_code >= 0;
                    const int out = valid ? out_code : -1 - out_code;
                    float* img = it.images + (size_t)out * w2;
                    const uint32_t* a = acc + g * (w2 + 4);
                    if ((w2 & 3) == 0 && ((reinterpret_cast<uintptr_t>(img) & 15) == 0)) {
                        for (int i = tid; i < w2 / 4; i += kBlock) {
                            const uint4 q = reinterpret_cast<const uint4*>(a)[i];
                            f32x4 f;
                            f[0] = (float)q.x * (1.0f / 65536.0f);
                            f[1] = (float)q.y * (1.0f / 65536.0f);
                            f[2] = (float)q.z * (1.0f / 65536.0f);
                            f[3] = (float)q.w * (1.0f / 65536.0f);
                            __builtin_nontemporal_store(f, reinterpret_cast<f32x4*>(img) + i);
                        }
                    } else {
                        for (int i = tid; i < w2; i += kBlock)
                            __builtin_nontemporal_store((float)a[i] * (1.0f / 65536.0f), img + i);
                    }
                    if (tid == 0) {
                        it.counts[out] = valid ? c : 0xFFFFFFFFu;
                        if (valid) my_support += c; else ++my_invalid;
                    }
                    if (valid && c >= d.ovf_limit) redo_mask |= 1 << g;
                }
                // ---- rare: an image with >= 65536 pairs may have wrapped a bin ----
                if (redo_mask) {
                    for (int g = 0; g < ng; ++g) {
                        if (!(redo_mask & (1 << g))) continue;
                        __syncthreads();
                        unsigned long long* acc64 = reinterpret_cast<unsigned long long*>(acc);
                        for (int i = tid; i < w2; i += kBlock) acc64[i] = 0ull;
                        __syncthreads();
                        uint32_t c1[1] = {0};
                        const ImgInfo inf = s_info[cur + g];
                        GroupImg one;
                        one.px = rfl(inf.px); one.py = rfl(inf.py); one.pz = rfl(inf.pz);
                        one.nx = rfl(inf.nx); one.ny = rfl(inf.ny); one.nz = rfl(inf.nz);
                        if (p.mode == SI_BIN_BILINEAR)
                            candidate_pass<SI_BIN_BILINEAR, 1, unsigned long long>(
                                sc, p, &one, 1, acc64, s_row_start, s_row_pref, n_rows, c1);
                        else
                            candidate_pass<SI_BIN_CEIL, 1, unsigned long long>(
                                sc, p, &one, 1, acc64, s_row_start, s_row_pref, n_rows, c1);
                        __syncthreads();
                        const int out = s_info[cur + g].out;
                        float* img = it.images + (size_t)out * w2;
                        for (int i = tid; i < w2; i += kBlock)
                            img[i] = (float)acc64[i] * (1.0f / 65536.0f);
                        if (tid == 0) ++my_overflow;
                    }
                }
                __syncthreads();
                if (EMU) {
                    // emulated heterogeneous workers: every emu_every-th
                    // workgroup, after each group, spends emu_extra times the
                    // group's own time more, so it runs (1 + emu_extra) times
                    // slower -- idling (its compute unit free for others) or
                    // with every thread spinning on arithmetic (its compute
                    // unit kept busy); its images do not change
                    if (rfl(s_slow)) {
                        if (tid == 0) {
                            const uint64_t t1 = wall_clock64();
                            s_until = t1 + (uint64_t)((float)(t1 - s_m.t_group) * d.emu_extra);
                        }
                        if (d.emu_busy) {
                            __syncthreads();
                            const uint64_t until = s_until;
                            float v = (float)tid;
                            while (wall_clock64() < until) {
#pragma unroll
                                for (int i = 0; i < 32; ++i) v = fmaf(v, 0.999f, 0.5f);
                            }
                            __asm__ volatile("" ::"v"(v));
                        } else if (tid == 0) {
                            const uint64_t until = s_until;
                            while (wall_clock64() < until) __builtin_amdgcn_s_sleep(4);
                        }
                    }
                    // AF: the group's time per image is one sample of this
                    // workgroup's iteration time (Welford's update)
                    if (tid == 0) {
                        const uint64_t t1 = wall_clock64();
                        const double x = ((double)(t1 - s_m.t_group) + 0.5) / (double)ng;
                        s_m.t_group = t1;
                        s_m.af_n += 1.0;
                        const double dlt = x - s_m.af_mean;
                        s_m.af_mean += dlt / s_m.af_n;
                        s_m.af_m2 += dlt * (x - s_m.af_mean);
                    }
                }
                cur += ng;
            }
        }
        if (EMU && d.rule && tid == 0) {
            // publish this workgroup's measurements for the next claims
            if (d.rule == SI_SCHED_AWF) {
                const double dt = (double)(wall_clock64() - s_m.t_chunk) + 0.5;
                const int k = ++s_m.aw_k;
                s_m.aw_a += (double)k * (double)(c_end - c_start);
                s_m.aw_b += (double)k * dt;
                const double rate = s_m.aw_a / s_m.aw_b;
                atomicAdd(&d.adapt[0], rate - s_m.aw_rate);
                if (k == 1) atomicAdd(&d.adapt[2], 1.0);
                s_m.aw_rate = rate;
            } else if (d.rule == SI_SCHED_AF && s_m.af_n >= 2.0) {
                const double c1 = 1.0 / s_m.af_mean;
                const double c2 = s_m.af_m2 / (s_m.af_n - 1.0) / s_m.af_mean;
                atomicAdd(&d.adapt[0], c1 - s_m.af_c1);
                atomicAdd(&d.adapt[1], c2 - s_m.af_c2);
                if (!s_m.af_meas) atomicAdd(&d.adapt[2], 1.0);
                s_m.af_meas = 1;
                s_m.af_c1 = c1;
                s_m.af_c2 = c2;
            }
        }
    }

    if (tid == 0) {
        if (d.stat_tested && my_tested) atomicAdd(d.stat_tested, my_tested);
        if (d.stat_support && my_support) atomicAdd(d.stat_support, my_support);
        if (d.stat_invalid && my_invalid) atomicAdd(d.stat_invalid, my_invalid);
        if (d.err_flag && my_invalid) atomicOr(d.err_flag, 1u);
        if (d.stat_overflow && my_overflow) atomicAdd(d.stat_overflow, my_overflow);
        if (EMU && d.stat_chunks && s_m.claims) atomicAdd(d.stat_chunks, s_m.claims);
        if (d.wg_ns) d.wg_ns[blockIdx.x] = (unsigned long long)(wall_clock64() - t_begin);
        if (d.dynamic) {
            // the last workgroup to finish leaves the counter at zero for the next launch
            __threadfence();
            const uint32_t done = atomicAdd(d.counter + 1, 1u);
            if (done == gridDim.x - 1) {
                atomicExch(d.counter, 0u);
                atomicExch(d.counter + 1, 0u);
                if (EMU && d.rule) atomicExch(d.counter + 2, 0u);
            }
        }
    }
}

size_t spin_lds_bytes(int max_w2, int group) {
    const int slots = group < 2 ? 2 : group;  // room for one 64-bit image
    return (size_t)slots * (size_t)(max_w2 + 4) * sizeof(uint32_t) + 16;
}

// Workgroups of k_spin that one CU holds at once: the occupancy calculator's
// answer, capped by the CU's LDS counted in allocation blocks of 1,280 bytes.
// The calculator alone over-counts on gfx950: 32,384 bytes per workgroup fit
// four to a 160 KB CU, not five (the fifth workgroup of every CU only starts
// when another ends), while 30,848 bytes fit five; 1,280-byte blocks
// reproduce both.
int spin_max_wg_per_cu(int max_w2, int group) {
    const size_t dyn = spin_lds_bytes(max_w2, group);
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, reinterpret_cast<const void*>(k_spin<false>), kBlock, dyn);
    if (e != hipSuccess || n < 1) n = 1;
    hipFuncAttributes fa;
    int dev = 0, cu_lds = 0;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k_spin<false>)) == hipSuccess &&
        hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cu_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
            hipSuccess &&
        cu_lds > 0) {
        constexpr size_t kLdsBlock = 1280;
        const size_t per_wg = (fa.sharedSizeBytes + dyn + kLdsBlock - 1) / kLdsBlock * kLdsBlock;
        n = std::max(1, std::min(n, (int)((size_t)cu_lds / per_wg)));
    }
    return n;
}

}  // namespace si

// The sticky invalid-index flag, one copy per device: word 0 is set by any
// generation launch that meets an oriented index outside [0, M); word 1
// receives it when it is read and cleared.
static __device__ uint32_t invalid_seen[2];

namespace si {

namespace {

std::mutex g_flag_mu;
std::map<int, uint32_t*> g_flag;  // device -> address of invalid_seen

hipError_t invalid_flag(uint32_t** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_flag_mu);
    auto it = g_flag.find(dev);
    if (it == g_flag.end()) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(invalid_seen));
        if (e != hipSuccess) return e;
        it = g_flag.emplace(dev, static_cast<uint32_t*>(p)).first;
    }
    *out = it->second;
    return hipSuccess;
}

__global__ void k_take_flag(uint32_t* f) {
    if (threadIdx.x == 0) f[1] = atomicExch(f, 0u);
}

}  // namespace

hipError_t launch_spin(const LaunchDesc& d, int n_wg, hipStream_t s) {
    LaunchDesc dd = d;
    if (!dd.err_flag) {
        const hipError_t e = invalid_flag(&dd.err_flag);
        if (e != hipSuccess) return e;
    }
    const size_t lds = spin_lds_bytes(dd.max_w2, dd.group);
    if (dd.emu_every > 0 || dd.rule != 0)
        hipLaunchKernelGGL(k_spin<true>, dim3(n_wg), dim3(kBlock), lds, s, dd);
    else
        hipLaunchKernelGGL(k_spin<false>, dim3(n_wg), dim3(kBlock), lds, s, dd);
    return hipGetLastError();
}

hipError_t take_invalid_flag(hipStream_t s, uint32_t* seen) {
    uint32_t* f = nullptr;
    hipError_t e = invalid_flag(&f);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_take_flag, dim3(1), dim3(64), 0, s, f);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(seen, f + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

}  // namespace si
