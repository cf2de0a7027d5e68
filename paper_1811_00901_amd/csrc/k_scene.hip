// Scene-building kernels: bounding box, cell binning, exclusive scan and the
// scatter of the oriented points (Section 2.1: OP, positions with normals)
// into a cell-sorted structure-of-arrays of 32-byte records.  The cell of a
// point is floor((x - origin) / h) per axis, evaluated in double precision so
// that the conservative culling in the spin kernel can reproduce cell
// boundaries exactly.
#include "scene_build.h"

namespace si {

namespace {

constexpr int kScanTile = 2048;        // elements per scan tile (256 threads x 8)
constexpr int kBBoxBlocks = 1024;

// Block-wide min/max of the finite coordinates of points first, first +
// stride, ... < M into out6 (lo xyz, hi xyz).
__device__ __forceinline__ void bbox_block(const float* __restrict__ xyz, int64_t M,
                                           int64_t first, int64_t stride, float* __restrict__ out6) {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = first; i < M; i += stride) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = xyz[3 * i + a];
            if (isfinite(v)) {
                lo[a] = fminf(lo[a], v);
                hi[a] = fmaxf(hi[a], v);
            }
        }
    }
    __shared__ float s[6][256];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + off]);
                s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + off]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) out6[threadIdx.x] = s[threadIdx.x][0];
}

// Block-wide reduction of n partial boxes (6 floats each) into out6.
__device__ __forceinline__ void bbox_reduce(const float* __restrict__ part, int64_t n,
                                            float* __restrict__ out6) {
    __shared__ float s[6][256];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = threadIdx.x; i < n; i += 256) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = fminf(v[a], part[i * 6 + a]);
            v[3 + a] = fmaxf(v[3 + a], part[i * 6 + 3 + a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) s[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + off]);
                s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + off]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) out6[threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_bbox_partial(const float* __restrict__ xyz, int64_t M,
                                                      float* __restrict__ part) {
    bbox_block(xyz, M, blockIdx.x * (int64_t)blockDim.x + threadIdx.x,
               (int64_t)gridDim.x * blockDim.x, part + blockIdx.x * 6);
}

__global__ void __launch_bounds__(256) k_bbox_final(const float* __restrict__ part, int n,
                                                    float* __restrict__ out6) {
    bbox_reduce(part, n, out6);
}

// Largest i < n with off[i] <= t (off ascending, off[0] <= t).
__device__ __forceinline__ int find_item(const int64_t* off, int n, int64_t t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Item of element t, for blocks of consecutive elements: the search for the
// block's first element is the same in every lane (its loads are uniform),
// and each thread then steps over the few segment ends inside the block.
__device__ __forceinline__ int find_item_block(const int64_t* off, int n, int64_t t) {
    int s = find_item(off, n, (int64_t)blockIdx.x * blockDim.x);
    while (s + 1 < n && off[s + 1] <= t) ++s;
    return s;
}

// Partial boxes of many scenes: block b works for scene s with
// blk_off[s] <= b < blk_off[s+1], striding over that scene's points.
__global__ void __launch_bounds__(256) k_bbox_partial_multi(const BuildItem* __restrict__ items,
                                                            const int64_t* __restrict__ blk_off,
                                                            int n, float* __restrict__ part) {
    const int s = find_item(blk_off, n, blockIdx.x);
    const int64_t lb = blockIdx.x - blk_off[s], nb = blk_off[s + 1] - blk_off[s];
    bbox_block(items[s].xyz, items[s].M, lb * blockDim.x + threadIdx.x, nb * blockDim.x,
               part + blockIdx.x * 6);
}

// One block per scene reduces its partial boxes.
__global__ void __launch_bounds__(256) k_bbox_final_multi(const int64_t* __restrict__ blk_off,
                                                          const float* __restrict__ part,
                                                          float* __restrict__ out6) {
    const int s = blockIdx.x;
    bbox_reduce(part + blk_off[s] * 6, blk_off[s + 1] - blk_off[s], out6 + 6 * s);
}

// Sort key of a point: cell * kSubX + the quarter of the cell along x,
// floor(kSubX t) - kSubX floor(t) for t = (x - origin) / h.
__device__ __forceinline__ int key_of_point(const GridDesc& g, float x, float y, float z) {
    const float v[3] = {x, y, z};
    int c[3];
    int sub = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = ((double)v[a] - g.origin[a]) / g.h;
        const double t = floor(u);
        // non-finite coordinates (never in support of anything) go to cell 0
        const bool ok = t >= 0.0 && t < (double)g.dims[a];
        c[a] = ok ? (int)t : 0;
        if (a == 0 && ok) sub = min(max((int)(floor(u * kSubX) - t * kSubX), 0), kSubX - 1);
    }
    return ((c[2] * g.dims[1] + c[1]) * g.dims[0] + c[0]) * kSubX + sub;
}

// Rank of this lane's point among the points of its key: one atomic per run
// of consecutive lanes with the same key (points in mesh order share cells,
// so a wave holds few runs), the run's lanes numbered from the base that
// atomic returns.  `ok` lanes form a prefix of the wave; every lane calls.
__device__ __forceinline__ int32_t rank_in_key(bool ok, int k, int32_t* counter_of_k) {
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(k, 1, 64);
    const bool start = ok && (lane == 0 || prev != k);
    const uint64_t starts = __builtin_amdgcn_ballot_w64(start);
    const uint64_t n_ok = (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(ok));
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);  // lanes 0..lane
    const uint64_t mine = starts & upto;
    const int run0 = mine ? 63 - __builtin_clzll(mine) : 0;  // this run's first lane
    const uint64_t later = starts & ~upto;
    const int run1 = later ? __builtin_ctzll(later) : (int)n_ok;  // the next run's
    int base = 0;
    if (start) base = atomicAdd(counter_of_k, run1 - run0);
    base = __shfl(base, run0, 64);
    return base + (lane - run0);
}

__global__ void __launch_bounds__(256) k_bin_points(const float* __restrict__ xyz, int64_t M,
                                                    GridDesc g, int32_t* __restrict__ key_of,
                                                    int32_t* __restrict__ rank,
                                                    int32_t* __restrict__ counts) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool ok = i < M;
    int k = -1;
    if (ok) {
        k = key_of_point(g, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
        key_of[i] = k;
    }
    const int32_t r = rank_in_key(ok, k, counts + (ok ? k : 0));
    if (ok) rank[i] = r;
}

// Tile sums of the input.
template <typename T>
__global__ void __launch_bounds__(256) k_scan_tiles(const T* __restrict__ in, int64_t n,
                                                    T* __restrict__ tile_sum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanTile / 256; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        if (i < n) s += in[i];
    }
    __shared__ T red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = red[0];
}

// Exclusive block scan of 256 values (four waves); returns the exclusive
// prefix, *total.  Each wave scans with shuffles; the four wave totals meet
// in s (at least 4 entries), two barriers in all.
template <typename T>
__device__ T block_excl_scan(T v, T* s, T* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) s[w] = x;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T t = s[k];
        if (k < w) before += t;
        all += t;
    }
    __syncthreads();  // s may be reused
    *total = all;
    return before + x - v;
}

// Exclusive scan of the tile sums in place (one workgroup).
template <typename T>
__global__ void __launch_bounds__(256) k_scan_tile_sums(T* __restrict__ t, int64_t n_tiles) {
    __shared__ T s[256];
    const int64_t per = (n_tiles + 255) / 256;
    const int64_t b = threadIdx.x * per;
    T sum = 0;
    for (int64_t k = 0; k < per; ++k)
        if (b + k < n_tiles) sum += t[b + k];
    T total;
    T run = block_excl_scan(sum, s, &total);
    for (int64_t k = 0; k < per; ++k) {
        if (b + k < n_tiles) {
            const T v = t[b + k];
            t[b + k] = run;
            run += v;
        }
    }
}

// Exclusive scan of each tile plus its offset; out[n] = total.
template <typename T>
__global__ void __launch_bounds__(256) k_scan_apply(const T* __restrict__ in, int64_t n,
                                                    const T* __restrict__ tile_off,
                                                    T* __restrict__ out) {
    __shared__ T s[256];
    constexpr int PER = kScanTile / 256;  // consecutive elements per thread
    constexpr int VEC = 16 / sizeof(T);   // elements per 16-byte access
    static_assert(PER % VEC == 0, "whole 16-byte accesses per thread");
    typedef __attribute__((ext_vector_type(VEC))) T vec_t;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * PER;
    // whole 16-byte accesses where the thread's elements are all in range
    // and both addresses are 16-byte aligned (callers' arrays need not be)
    const bool whole = base + PER <= n &&
                       ((reinterpret_cast<uintptr_t>(in + base) |
                         reinterpret_cast<uintptr_t>(out + base)) & 15) == 0;
    T v[PER];
    T sum = 0;
    if (whole) {
#pragma unroll
        for (int k = 0; k < PER; k += VEC) {
            const vec_t x = *reinterpret_cast<const vec_t*>(in + base + k);
#pragma unroll
            for (int j = 0; j < VEC; ++j) v[k + j] = x[j];
        }
    } else {
#pragma unroll
        for (int k = 0; k < PER; ++k) v[k] = (base + k < n) ? in[base + k] : 0;
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) sum += v[k];
    T total;
    T run = block_excl_scan(sum, s, &total) + tile_off[blockIdx.x];
    if (whole) {
#pragma unroll
        for (int k = 0; k < PER; k += VEC) {
            vec_t x;
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                x[j] = run;
                run += v[k + j];
            }
            *reinterpret_cast<vec_t*>(out + base + k) = x;
        }
    } else {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (base + k < n) out[base + k] = run;
            run += v[k];
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = tile_off[blockIdx.x] + total;
}

__global__ void __launch_bounds__(256) k_scatter(const float* __restrict__ xyz,
                                                 const float* __restrict__ nrm, int64_t M,
                                                 const int32_t* __restrict__ key_of,
                                                 const int32_t* __restrict__ rank,
                                                 const int32_t* __restrict__ sub_start,
                                                 float4* __restrict__ pos, float4* __restrict__ nr,
                                                 int32_t* __restrict__ inv) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int k = key_of[i];
    const int s = sub_start[k] + rank[i];
    pos[s] = make_float4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], __int_as_float(k / kSubX));
    nr[s] = make_float4(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2], __int_as_float((int)i));
    inv[i] = s;
}

// Batched build: point t of the concatenation, scene s = its segment.
__global__ void __launch_bounds__(256) k_bin_points_multi(const BuildItem* __restrict__ items,
                                                          const int64_t* __restrict__ pt_off,
                                                          int n, int64_t total_M,
                                                          int32_t* __restrict__ key_of,
                                                          int32_t* __restrict__ rank,
                                                          int32_t* __restrict__ counts) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool ok = t < total_M;
    int k = -1;  // the key in the concatenated key space
    if (ok) {
        const int s = find_item_block(pt_off, n, t);
        const BuildItem& it = items[s];
        const int64_t i = t - pt_off[s];
        const int kk = key_of_point(it.g, it.xyz[3 * i], it.xyz[3 * i + 1], it.xyz[3 * i + 2]);
        key_of[t] = kk;
        k = (int)(it.key_base + kk);
    }
    const int32_t r = rank_in_key(ok, k, counts + (ok ? k : 0));
    if (ok) rank[t] = r;
}

// sub_start of every scene from the scan of the concatenated counts:
// entry j of scene s is gscan[key_base + j] - gscan[key_base].
__global__ void __launch_bounds__(256) k_sub_start_multi(const BuildItem* __restrict__ items,
                                                         const int64_t* __restrict__ sub_off,
                                                         int n, int64_t total,
                                                         const int32_t* __restrict__ gscan) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int s = find_item_block(sub_off, n, t);
    const int64_t kb = items[s].key_base;
    items[s].sub_start[t - sub_off[s]] = gscan[kb + (t - sub_off[s])] - gscan[kb];
}

__global__ void __launch_bounds__(256) k_scatter_multi(const BuildItem* __restrict__ items,
                                                       const int64_t* __restrict__ pt_off, int n,
                                                       int64_t total_M,
                                                       const int32_t* __restrict__ key_of,
                                                       const int32_t* __restrict__ rank,
                                                       const int32_t* __restrict__ gscan) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= total_M) return;
    const int s = find_item_block(pt_off, n, t);
    const BuildItem& it = items[s];
    const int64_t i = t - pt_off[s];
    const int k = key_of[t];
    const int sp = gscan[it.key_base + k] - gscan[it.key_base] + rank[t];
    it.pos[sp] = make_float4(it.xyz[3 * i], it.xyz[3 * i + 1], it.xyz[3 * i + 2],
                             __int_as_float(k / kSubX));
    it.nr[sp] = make_float4(it.nrm[3 * i], it.nrm[3 * i + 1], it.nrm[3 * i + 2],
                            __int_as_float((int)i));
    it.inv[i] = sp;
}

__global__ void __launch_bounds__(256) k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Key (cell of the oriented point) and rank within its cell for each iteration.
__global__ void __launch_bounds__(256) k_order_keys(const int32_t* __restrict__ oriented, int64_t N,
                                                    const int32_t* __restrict__ inv, int64_t M,
                                                    int32_t* __restrict__ key,
                                                    int32_t* __restrict__ rank,
                                                    int32_t* __restrict__ counts) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int o = oriented[i];
    const int c = (o >= 0 && o < M) ? inv[o] : 0;
    key[i] = c;
    rank[i] = atomicAdd(counts + c, 1);
}

__global__ void __launch_bounds__(256) k_order_scatter(const int32_t* __restrict__ key,
                                                       const int32_t* __restrict__ rank, int64_t N,
                                                       const int32_t* __restrict__ starts,
                                                       int32_t* __restrict__ perm) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    perm[starts[key[i]] + rank[i]] = (int32_t)i;
}

__global__ void __launch_bounds__(256) k_order_keys_multi(const Item* __restrict__ items,
                                                          const int64_t* __restrict__ item_off,
                                                          const int64_t* __restrict__ key_base,
                                                          int n_items, int64_t total_N,
                                                          int32_t* __restrict__ key,
                                                          int32_t* __restrict__ rank,
                                                          int32_t* __restrict__ counts) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= total_N) return;
    const int i = find_item_block(item_off, n_items, t);
    const Item& it = items[i];
    const int o = it.oriented[t - item_off[i]];
    const int c = (o >= 0 && o < it.scene.M) ? it.scene.inv[o] : 0;
    const int64_t k = key_base[i] + c;
    key[t] = (int32_t)k;
    rank[t] = atomicAdd(counts + k, 1);
}

__global__ void __launch_bounds__(256) k_order_scatter_multi(const int32_t* __restrict__ key,
                                                             const int32_t* __restrict__ rank,
                                                             const int64_t* __restrict__ item_off,
                                                             int n_items, int64_t total_N,
                                                             const int32_t* __restrict__ starts,
                                                             int32_t* __restrict__ perm) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= total_N) return;
    const int i = find_item_block(item_off, n_items, t);
    perm[starts[key[t]] + rank[t]] = (int32_t)(t - item_off[i]);
}

}  // namespace

hipError_t launch_cell_order_multi(const Item* items, const int64_t* item_off,
                                   const int64_t* key_base, int n_items, int64_t total_N,
                                   int64_t total_keys, int32_t* key, int32_t* rank,
                                   int32_t* counts, int32_t* starts, int32_t* tmp, int32_t* perm,
                                   hipStream_t s) {
    hipError_t e = launch_fill(counts, total_keys, 0, s);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((total_N + 255) / 256);
    hipLaunchKernelGGL(k_order_keys_multi, dim3(nb), dim3(256), 0, s, items, item_off, key_base,
                       n_items, total_N, key, rank, counts);
    e = launch_scan(counts, starts, total_keys, tmp, scan_tmp_elems(total_keys), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_order_scatter_multi, dim3(nb), dim3(256), 0, s, key, rank, item_off,
                       n_items, total_N, starts, perm);
    return hipGetLastError();
}

hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)nb), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_cell_order(const int32_t* oriented, int64_t N, const Scene& sc, int32_t* key,
                             int32_t* rank, int32_t* counts, int32_t* starts, int32_t* tmp,
                             int32_t* perm, hipStream_t s) {
    hipError_t e = launch_fill(counts, sc.M, 0, s);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_order_keys, dim3(nb), dim3(256), 0, s, oriented, N, sc.inv, sc.M, key,
                       rank, counts);
    e = launch_scan(counts, starts, sc.M, tmp, scan_tmp_elems(sc.M), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_order_scatter, dim3(nb), dim3(256), 0, s, key, rank, N, starts, perm);
    return hipGetLastError();
}

hipError_t launch_bbox(const float* xyz, int64_t M, float* out6, hipStream_t s) {
    // out6 holds 6 floats followed by scratch for kBBoxBlocks * 6 partials
    const int nb = (int)std::min<int64_t>(kBBoxBlocks, (M + 255) / 256);
    float* part = out6 + 8;
    hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(256), 0, s, xyz, M, part);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, s, part, nb, out6);
    return hipGetLastError();
}

hipError_t launch_bin_points(const float* xyz, int64_t M, const Scene& sc, int32_t* key_of,
                             int32_t* rank, int32_t* counts, hipStream_t s) {
    const GridDesc g = grid_of(sc);
    hipLaunchKernelGGL(k_bin_points, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, xyz, M,
                       g, key_of, rank, counts);
    return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

template <typename T>
static hipError_t scan_impl(const T* in, T* out, int64_t n, T* tmp, hipStream_t s) {
    const int64_t nt = (n + kScanTile - 1) / kScanTile;
    if (nt == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, reinterpret_cast<int32_t*>(out),
                           (int64_t)(sizeof(T) / 4), 0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_tiles<T>, dim3((unsigned)nt), dim3(256), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_tile_sums<T>, dim3(1), dim3(256), 0, s, tmp, nt);
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)nt), dim3(256), 0, s, in, n, tmp, out);
    return hipGetLastError();
}

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, int64_t,
                       hipStream_t s) {
    return scan_impl<int32_t>(in, out, n, tmp, s);
}

hipError_t launch_scan64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
    return scan_impl<int64_t>(in, out, n, tmp, s);
}

hipError_t launch_scatter(const float* xyz, const float* nrm, int64_t M, const int32_t* key_of,
                          const int32_t* rank, const int32_t* sub_start, Scene& sc,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, xyz, nrm,
                       M, key_of, rank, sub_start, sc.pos, sc.nrm, sc.inv);
    return hipGetLastError();
}

hipError_t launch_bbox_multi(const BuildItem* items, const int64_t* blk_off, int n,
                             int64_t total_blocks, float* part, float* out6, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bbox_partial_multi, dim3((unsigned)total_blocks), dim3(256), 0, s, items,
                       blk_off, n, part);
    hipLaunchKernelGGL(k_bbox_final_multi, dim3((unsigned)n), dim3(256), 0, s, blk_off, part,
                       out6);
    return hipGetLastError();
}

hipError_t launch_build_multi(const BuildItem* items, const int64_t* pt_off,
                              const int64_t* sub_off, int n, int64_t total_M, int64_t total_keys,
                              int32_t* key_of, int32_t* rank, int32_t* counts, int32_t* gscan,
                              int32_t* tmp, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipError_t e = launch_fill(counts, total_keys, 0, s);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((total_M + 255) / 256);
    hipLaunchKernelGGL(k_bin_points_multi, dim3(nb), dim3(256), 0, s, items, pt_off, n, total_M,
                       key_of, rank, counts);
    e = launch_scan(counts, gscan, total_keys, tmp, scan_tmp_elems(total_keys), s);
    if (e != hipSuccess) return e;
    const int64_t total_sub = total_keys + n;
    hipLaunchKernelGGL(k_sub_start_multi, dim3((unsigned)((total_sub + 255) / 256)), dim3(256), 0,
                       s, items, sub_off, n, total_sub, gscan);
    hipLaunchKernelGGL(k_scatter_multi, dim3(nb), dim3(256), 0, s, items, pt_off, n, total_M,
                       key_of, rank, gscan);
    return hipGetLastError();
}

}  // namespace si
