// Workloads next to spin-image generation, on gfx950.
//
// * Mesh resolution (si_mesh_resolution): the paper sets the bin size B as a
//   factor of the mesh resolution (Section 2.1, notation table); read as the
//   mean distance from a point to its nearest other point.  One thread per
//   query point searches the scene's cell grid in shells of cells at
//   Chebyshev distance r = 0, 1, 2, ... from its own cell; every point not yet
//   searched is farther than r h, so the search stops as soon as the best
//   distance is within r h (exact, whatever the spacing).  Inside a shell,
//   cells and their quarter runs along x that lie farther than the best
//   distance so far are skipped.
// * Spin-image correlation (si_correlate): the normalised linear correlation
//   coefficient of two images' bins, the comparison by which spin images are
//   matched in object recognition (Johnson and Hebert, cited by the paper):
//       R = (N sum pq - sum p sum q) / sqrt((N sum p^2 - (sum p)^2)(N sum q^2 - (sum q)^2))
//   over N = W^2 bins, for every pair of two image sets.  sum pq over all
//   pairs is a dense contraction (n_a x n_b x N): it runs on the matrix cores
//   with fp16 operands and fp32 accumulation.  Each image is first scaled by
//   its largest bin (R does not change under a positive scale) and rounded to
//   fp16; its sums are taken from the rounded values, so R is the exact
//   correlation of the rounded images up to fp32 accumulation.
// * Normal estimation (si_estimate_normals), for points without normals
//   (the paper's oriented points come with them): the eigenvector of the
//   smallest eigenvalue of the covariance of each point's neighbours within a
//   radius, signed away from a viewpoint.
#include "si_internal.h"

#include <math.h>
#include <string.h>

#include <algorithm>

namespace si {
namespace {

// ------------------------------------------------------ mesh resolution --
__global__ void __launch_bounds__(256) k_nn(SceneView sc, const int32_t* __restrict__ idx,
                                            int64_t n, float* __restrict__ nn,
                                            double* __restrict__ acc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double mine = 0.0;
    double bad = 0.0;
    if (i < n) {
        const int o = idx ? idx[i] : (int)i;
        if (o < 0 || o >= sc.M) {
            if (nn) nn[i] = __int_as_float(0x7fc00000);
            bad = 1.0;
        } else {
            const int sp = sc.inv[o];
            const float4 p = sc.pos[sp];
            const int cell = __float_as_int(p.w);
            const int c0 = cell % sc.dims[0];
            const int c1 = (cell / sc.dims[0]) % sc.dims[1];
            const int c2 = cell / (sc.dims[0] * sc.dims[1]);
            const int rmax = max(max(max(c0, sc.dims[0] - 1 - c0), max(c1, sc.dims[1] - 1 - c1)),
                                 max(c2, sc.dims[2] - 1 - c2));
            // boxes in float32 relative to the grid's origin: a box is skipped
            // only when it is farther than the best distance by more than
            // eps, many ulp of the largest coordinate (as the spin kernel's
            // row culling), so rounding never skips a nearer point
            const float h = (float)sc.h, hq = (float)(sc.h / kSubX);
            float mag = 0.0f;
            for (int a = 0; a < 3; ++a)
                mag = fmaxf(mag, fabsf(sc.origin[a]) + (float)sc.dims[a] * h);
            const float eps = 2e-6f * mag + 1e-6f;
            const float ox = p.x - sc.origin[0], oy = p.y - sc.origin[1], oz = p.z - sc.origin[2];
            // distance from the point to [lo, lo + w] along one axis, less eps
            auto gap = [eps](float o, float lo, float w) {
                return fmaxf(0.0f, fmaxf(lo - o, o - (lo + w)) - eps);
            };
            const int qp = min(max((int)floorf((ox - (float)c0 * h) / hq), 0), kSubX - 1);
            float best = __int_as_float(0x7f800000);
            for (int r = 0; r <= rmax; ++r) {
                for (int dz = -r; dz <= r; ++dz) {
                    const int z = c2 + dz;
                    if (z < 0 || z >= sc.dims[2]) continue;
                    const float gz = gap(oz, (float)z * h, h);
                    for (int dy = -r; dy <= r; ++dy) {
                        const int y = c1 + dy;
                        if (y < 0 || y >= sc.dims[1]) continue;
                        const float gy = gap(oy, (float)y * h, h);
                        const float dyz = fmaf(gz, gz, gy * gy);
                        if (dyz > best) continue;
                        // on the shell: all of x when y or z is at distance r
                        const bool face = (dz == -r || dz == r || dy == -r || dy == r);
                        for (int dx = -r; dx <= r; dx += (face || r == 0) ? 1 : 2 * r) {
                            const int x = c0 + dx;
                            if (x < 0 || x >= sc.dims[0]) continue;
                            const int key = ((z * sc.dims[1] + y) * sc.dims[0] + x) * kSubX;
                            // the cell's quarter runs along x, nearest first
                            for (int t = 0; t < kSubX; ++t) {
                                const int q = x < c0 ? kSubX - 1 - t
                                              : x > c0 ? t
                                              : (t == 0 ? qp : (t - 1 < qp ? t - 1 : t));
                                const float gx = gap(ox, (float)x * h + (float)q * hq, hq);
                                if (fmaf(gx, gx, dyz) > best) continue;
                                const int a = sc.sub_start[key + q], b = sc.sub_start[key + q + 1];
                                for (int j = a; j < b; ++j) {
                                    if (j == sp) continue;
                                    const float4 w = sc.pos[j];
                                    const float ex = w.x - p.x, ey = w.y - p.y, ez = w.z - p.z;
                                    best = fminf(best, fmaf(ez, ez, fmaf(ey, ey, ex * ex)));
                                }
                            }
                        }
                    }
                }
                // every point outside shells 0..r lies more than r h away
                const double lim = (double)r * sc.h * (1.0 - 1e-6);
                if ((double)best <= lim * lim) break;
            }
            const float d = sqrtf(best);
            if (nn) nn[i] = d;
            mine = (double)d;
        }
    }
    // block sums of the distances (and of invalid indices), one atomic each
    __shared__ double s_sum[256 / 64], s_bad[256 / 64];
    for (int off = 32; off > 0; off >>= 1) {
        mine += __shfl_xor(mine, off, 64);
        bad += __shfl_xor(bad, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_sum[threadIdx.x >> 6] = mine;
        s_bad[threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0, u = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            t += s_sum[w];
            u += s_bad[w];
        }
        if (t != 0.0) atomicAdd(acc, t);
        if (u != 0.0) atomicAdd(acc + 1, u);
    }
}

// ----------------------------------------------------------- correlation --
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 256, kTN = 128;  // A rows and B rows (images) per workgroup tile
constexpr int kWavesM = 4, kWavesN = 2;  // waves per tile, each 64 x 64
constexpr int kGemmThreads = 64 * kWavesM * kWavesN;
constexpr int kBK = 32;               // K (bins) per LDS stage: one MFMA depth
constexpr int kSuperM = 8, kSuperN = 8;  // tiles one XCD runs at once (two per CU)

// One wave per image: scale by the largest bin, round to fp16 into a row of
// Kp halves (zero beyond N), and keep the rounded image's sum s and
// rs = 1 / sqrt(N sum h^2 - s^2) (0 when the image has no variance).
__global__ void __launch_bounds__(256) k_corr_prep(const float* __restrict__ X, int64_t n, int N,
                                                   int Kp, _Float16* __restrict__ H,
                                                   float2* __restrict__ stats) {
    const int lane = threadIdx.x & 63;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (row >= n) return;
    const float* x = X + row * (int64_t)N;
    float mx = 0.0f;
    for (int k = lane; k < N; k += 64) mx = fmaxf(mx, fabsf(x[k]));
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    const float inv = mx > 0.0f ? 1.0f / mx : 1.0f;
    double s = 0.0, q = 0.0;
    _Float16* h = H + row * (int64_t)Kp;
    for (int k = lane; k < Kp; k += 64) {
        const _Float16 v = (_Float16)(k < N ? x[k] * inv : 0.0f);
        h[k] = v;
        const double f = (double)(float)v;
        s += f;
        q += f * f;
    }
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        q += __shfl_xor(q, off, 64);
    }
    if (lane == 0) {
        const double var = (double)N * q - s * s;
        stats[row] = make_float2((float)s, var > 0.0 ? (float)(1.0 / sqrt(var)) : 0.0f);
    }
}

// Order-preserving 64-bit key of (R, j): larger R first, then smaller j.
__device__ __forceinline__ unsigned long long best_key(float r, int j) {
    const uint32_t b = __float_as_uint(r);
    const uint32_t o = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((unsigned long long)o << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)j);
}

// Largest x, and smallest i, over the 16 lanes of each DPP row; every lane
// receives the result (swap neighbours, swap pairs, mirror each half, mirror
// the row).
__device__ __forceinline__ float row16_max(float x) {
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x141, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x140, 0xF, 0xF, false)));
    return x;
}
__device__ __forceinline__ int row16_min(int i) {
    i = min(i, __builtin_amdgcn_mov_dpp(i, 0xB1, 0xF, 0xF, false));
    i = min(i, __builtin_amdgcn_mov_dpp(i, 0x4E, 0xF, 0xF, false));
    i = min(i, __builtin_amdgcn_mov_dpp(i, 0x141, 0xF, 0xF, false));
    i = min(i, __builtin_amdgcn_mov_dpp(i, 0x140, 0xF, 0xF, false));
    return i;
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// R for a 256 x 128 tile of (A image, B image) pairs.  Eight waves, each a
// 64 x 64 part as 4 x 4 products of 16 x 16 (v_mfma_f32_16x16x32_f16: lane l
// holds row l % 16 of the A operand and of B's image at K = 8 (l / 16) .. + 7,
// and receives column l % 16, rows 4 (l / 16) .. + 3 of the result); two
// workgroups per compute unit.
//
// Operands move from global memory straight into LDS (global_load_lds_dwordx4,
// no registers in between), 32 bins per stage, into a ring of three stages:
// while the products of stage s run, the loads of stages s + 1 and s + 2 are
// in flight.  A stage is 24 groups of 16 rows x 64 bytes, three per wave; in
// a group, lane l fills bytes 16 l .. 16 l + 15, i.e. row l / 4, slot l % 4,
// and loads the chunk (l % 4) ^ ((row / 2) % 4) of that row, so that each
// row's four 16-byte chunks sit XOR-swizzled by bits 1-2 of the row.  Taking
// a ds_read_b128 as eight lanes (128 bytes over 32 banks) per pass, a
// fragment read's pass covers eight consecutive rows at one logical chunk,
// in 16-byte slots 4 (row % 2) + chunk ^ ((row / 2) % 4): all distinct.
// (Swizzled by the row's low bits, rows r and r + 2 shared banks; by bits
// 2-3, right for 16 lanes per pass, it ran no faster: the measured order
// matches the eight-lane model.)  Each iteration waits on
// vmcnt for this wave's loads of stage s only, then a barrier (with no
// memory fence, which would wait for every load in flight) makes all waves'
// loads of stage s visible and guarantees that the stage read two iterations
// ago is no longer read, before its slot receives stage s + 2.  Rows past
// the end of A or B load the last row (their results are never used), so
// the loads need no branches.
//
// Tiles are numbered in super-tiles of 8 x 8: the 64 workgroups one XCD runs
// at once (workgroup ids congruent mod 8) share 8 A bands and 8 B bands in
// that XCD's L2.  Each row's best column is reduced over its 16 lanes with
// DPP and merged across tiles by a 64-bit atomicMax.
__global__ void __launch_bounds__(kGemmThreads, 2)
    k_corr_gemm(const _Float16* __restrict__ HA, const _Float16* __restrict__ HB,
                const float2* __restrict__ SA, const float2* __restrict__ SB, int64_t n_a,
                int64_t n_b, int N, int Kp, int64_t tiles_m, int64_t tiles_n, int64_t super_n,
                float* __restrict__ Rout, unsigned long long* __restrict__ best) {
    constexpr int kWaves = kWavesM * kWavesN;
    constexpr int CPR = kBK / 8;                // 16-byte chunks per LDS row
    constexpr int kStage = (kTM + kTN) * kBK;   // halves per stage
    constexpr int kGroups = (kTM + kTN) / 16;   // 1 KB loads per stage
    constexpr int PW = kGroups / kWaves;        // ... per wave
    static_assert(kGroups % kWaves == 0 && PW < 16, "whole loads per wave, vmcnt field");
    __shared__ __attribute__((aligned(16))) _Float16 ring[3][kStage];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t L = blockIdx.x;
    const int64_t j = L >> 3;
    const int64_t s = (j / (kSuperM * kSuperN)) * 8 + (L & 7);
    const int i = (int)(j % (kSuperM * kSuperN));
    const int64_t tm = (s / super_n) * kSuperM + i / kSuperN;
    const int64_t tn = (s % super_n) * kSuperN + i % kSuperN;
    if (tm >= tiles_m || tn >= tiles_n) return;
    const int64_t m0 = tm * kTM, n0 = tn * kTN;
    const int wm = wave / kWavesN, wn = wave % kWavesN;
    const int r16 = lane & 15, kq = lane >> 4;
    auto off = [](int row, int ch) { return row * kBK + 8 * (ch ^ ((row >> 1) & (CPR - 1))); };
    // this lane's sources: groups wave, wave + 8, wave + 16 of the stage's
    // rows (A's 256, then B's 128)
    const int lr = lane >> 2;
    const int lch = (lane & 3) ^ ((lr >> 1) & 3);
    const _Float16* src[PW];
    int dst[PW];
#pragma unroll
    for (int k = 0; k < PW; ++k) {
        const int g = wave + kWaves * k;
        if (g < kTM / 16)
            src[k] = HA + min(m0 + 16 * g + lr, n_a - 1) * Kp + 8 * lch;
        else
            src[k] = HB + min(n0 + 16 * (g - kTM / 16) + lr, n_b - 1) * Kp + 8 * lch;
        dst[k] = 16 * g * kBK;
    }
    auto issue = [&](int st) {
        _Float16* r = ring[st % 3];
        const int k0 = st * kBK;
#pragma unroll
        for (int k = 0; k < PW; ++k)
            __builtin_amdgcn_global_load_lds((const glb_void_t*)(src[k] + k0),
                                             (lds_void_t*)(r + dst[k]), 16, 0, 0);
    };
    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
    const int n_st = Kp / kBK;
    issue(0);
    if (n_st > 1) issue(1);
    for (int st = 0; st < n_st; ++st) {
        // s_waitcnt immediates: vmcnt in bits 3:0, expcnt and lgkmcnt at their
        // maxima (no wait on them)
        if (st + 1 < n_st) __builtin_amdgcn_s_waitcnt(0x0F70 | PW);  // vmcnt(PW)
        else __builtin_amdgcn_s_waitcnt(0x0F70);                     // vmcnt(0)
        __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no LDS access moves across
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (st + 2 < n_st) issue(st + 2);
        const _Float16* As = ring[st % 3];
        const _Float16* Bs = As + kTM * kBK;
        h8 fb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            fb[t] = *reinterpret_cast<const h8*>(&Bs[off(wn * 64 + t * 16 + r16, kq)]);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const h8 fa = *reinterpret_cast<const h8*>(&As[off(wm * 64 + a * 16 + r16, kq)]);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fa, fb[b], acc[a][b], 0, 0, 0);
        }
    }
    // epilogue: R, optional store, and each row's best column in this tile
    const float fN = (float)N;
    float2 sb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t col = n0 + wn * 64 + b * 16 + r16;
        sb[b] = col < n_b ? SB[col] : make_float2(0.0f, 0.0f);
    }
    const float ninf = -__builtin_inff();
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = m0 + wm * 64 + a * 16 + 4 * kq + v;
            const bool row_ok = row < n_a;
            const float2 sa = row_ok ? SA[row] : make_float2(0.0f, 0.0f);
            float rb = ninf;
            int bb = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int64_t col = n0 + wn * 64 + b * 16 + r16;
                const float r = (fN * acc[a][b][v] - sa.x * sb[b].x) * sa.y * sb[b].y;
                if (Rout && row_ok && col < n_b) Rout[row * n_b + col] = r;
                // strictly larger: the lowest column wins ties (-0 equals +0)
                if (col < n_b && r > rb) {
                    rb = r;
                    bb = b;
                }
            }
            if (best) {
                // the 16 lanes of one row hold its columns of this wave
                const float m = row16_max(rb);
                const int c = row16_min(rb == m ? wn * 64 + bb * 16 + r16 : 0x7fffffff);
                if (r16 == 0 && row_ok && m > ninf)
                    atomicMax(best + row, best_key(m == 0.0f ? 0.0f : m, (int)(n0 + c)));
            }
        }
    }
}

__global__ void k_corr_best(const unsigned long long* __restrict__ best, int64_t n,
                            int32_t* __restrict__ idx, float* __restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long k = best[i];
    const uint32_t o = (uint32_t)(k >> 32);
    const uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    if (idx) idx[i] = (int32_t)(0xFFFFFFFFu - (uint32_t)k);
    if (r) r[i] = __uint_as_float(b);
}

size_t rup256(size_t b) { return (b + 255) & ~(size_t)255; }

// ------------------------------------------------------ normal estimation --
// Unit eigenvector of the smallest eigenvalue of the symmetric 3 x 3 matrix
// [[a00 a01 a02] [a01 a11 a12] [a02 a12 a22]]: the eigenvalue from the
// trigonometric closed form of the characteristic cubic, the vector as the
// longest cross product of two rows of A - l0 I (each row is orthogonal to
// it).  A multiple of the identity has no preferred direction: e_z.
__device__ void smallest_eigvec(double a00, double a01, double a02, double a11, double a12,
                                double a22, double n[3]) {
    const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
    const double q = (a00 + a11 + a22) / 3.0;
    const double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
    const double p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * p1;
    n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
    if (!(p2 > 0.0)) return;
    const double p = sqrt(p2 / 6.0);
    const double c00 = b00 / p, c11 = b11 / p, c22 = b22 / p;
    const double c01 = a01 / p, c02 = a02 / p, c12 = a12 / p;
    double r = 0.5 * (c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) +
                      c02 * (c01 * c12 - c11 * c02));
    r = fmin(1.0, fmax(-1.0, r));
    const double phi = acos(r) / 3.0;
    const double l0 = q + 2.0 * p * cos(phi + 2.0943951023931957);  // + 2 pi / 3
    const double r0[3] = {a00 - l0, a01, a02};
    const double r1[3] = {a01, a11 - l0, a12};
    const double r2[3] = {a02, a12, a22 - l0};
    auto cross = [](const double* u, const double* v, double* w) {
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
    };
    double c[3][3];
    cross(r0, r1, c[0]);
    cross(r0, r2, c[1]);
    cross(r1, r2, c[2]);
    int best = 0;
    double bn = -1.0;
    for (int k = 0; k < 3; ++k) {
        const double m = c[k][0] * c[k][0] + c[k][1] * c[k][1] + c[k][2] * c[k][2];
        if (m > bn) { bn = m; best = k; }
    }
    if (!(bn > 0.0)) return;
    const double inv = 1.0 / sqrt(bn);
    n[0] = c[best][0] * inv; n[1] = c[best][1] * inv; n[2] = c[best][2] * inv;
}

// One thread per point in the grid's sorted order (neighbouring threads share
// cells): the points within r among the 27 cells around it (cell edge >= r),
// their FP64 sums relative to the point, covariance about their centroid, the
// smallest-eigenvalue eigenvector signed away from the viewpoint, written at
// the point's original index.
__global__ void __launch_bounds__(256) k_normals(SceneView sc, float r, float vx, float vy,
                                                 float vz, float* __restrict__ out,
                                                 int32_t* __restrict__ counts) {
    const int sp = blockIdx.x * blockDim.x + threadIdx.x;
    if (sp >= sc.M) return;
    const float4 p = sc.pos[sp];
    const int o = __float_as_int(sc.nrm[sp].w);
    const float r2 = r * r;
    const int cell = __float_as_int(p.w);
    const int c0 = cell % sc.dims[0];
    const int c1 = (cell / sc.dims[0]) % sc.dims[1];
    const int c2 = cell / (sc.dims[0] * sc.dims[1]);
    double n = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    double sxx = 0.0, sxy = 0.0, sxz = 0.0, syy = 0.0, syz = 0.0, szz = 0.0;
    for (int z = max(c2 - 1, 0); z <= min(c2 + 1, sc.dims[2] - 1); ++z)
        for (int y = max(c1 - 1, 0); y <= min(c1 + 1, sc.dims[1] - 1); ++y) {
            const int x0 = max(c0 - 1, 0), x1 = min(c0 + 1, sc.dims[0] - 1);
            const int base = (z * sc.dims[1] + y) * sc.dims[0];
            // the cells x0..x1 of a row are one run of the sorted points
            const int a = sc.sub_start[(base + x0) * kSubX], b = sc.sub_start[(base + x1 + 1) * kSubX];
            for (int j = a; j < b; ++j) {
                const float4 q = sc.pos[j];
                const float dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
                if (fmaf(dz, dz, fmaf(dy, dy, dx * dx)) <= r2) {
                    const double ex = dx, ey = dy, ez = dz;
                    n += 1.0;
                    sx += ex; sy += ey; sz += ez;
                    sxx += ex * ex; sxy += ex * ey; sxz += ex * ez;
                    syy += ey * ey; syz += ey * ez; szz += ez * ez;
                }
            }
        }
    const double mx = sx / n, my = sy / n, mz = sz / n;
    double v[3];
    smallest_eigvec(sxx / n - mx * mx, sxy / n - mx * my, sxz / n - mx * mz, syy / n - my * my,
                    syz / n - my * mz, szz / n - mz * mz, v);
    const double s = v[0] * ((double)p.x - vx) + v[1] * ((double)p.y - vy) +
                     v[2] * ((double)p.z - vz);
    const double sg = s < 0.0 ? -1.0 : 1.0;
    out[3 * (int64_t)o] = (float)(sg * v[0]);
    out[3 * (int64_t)o + 1] = (float)(sg * v[1]);
    out[3 * (int64_t)o + 2] = (float)(sg * v[2]);
    if (counts) counts[o] = (int32_t)n;
}

}  // namespace
}  // namespace si

using namespace si;

extern "C" si_status si_mesh_resolution(const si_scene* scene, const int32_t* idx, int64_t n,
                                        float* nn_out, double* mean_out, void* hip_stream) {
    if (!scene) return fail(SI_E_INVALID, "scene is NULL");
    if (!mean_out) return fail(SI_E_INVALID, "mean_out is NULL");
    if (scene->M < 2) return fail(SI_E_INVALID, "a scene of one point has no nearest neighbour");
    if (!idx) n = scene->M;
    if (n <= 0 || n >= INT32_MAX) return fail(SI_E_INVALID, "n must be in [1, 2^31 - 1)");
    int cur = 0;
    SI_HIP(hipGetDevice(&cur));
    if (cur != scene->device) return fail(SI_E_INVALID, "scene lives on another device");
    hipStream_t s = (hipStream_t)hip_stream;
    double* acc = nullptr;
    SI_HIP(pool_alloc((void**)&acc, 2 * sizeof(double), s));
    hipError_t e = launch_fill(reinterpret_cast<int32_t*>(acc), 4, 0, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_nn, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           view_of(*scene), idx, n, nn_out, acc);
        e = hipGetLastError();
    }
    double h[2] = {0.0, 0.0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s);
    (void)hipFreeAsync(acc, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "mesh resolution");
    if (h[1] > 0.0) return fail(SI_E_INVALID, "idx holds indices outside [0, M)");
    *mean_out = h[0] / (double)n;
    return SI_OK;
}

extern "C" si_status si_correlate(const float* A, int64_t n_a, const float* B, int64_t n_b,
                                  int32_t n_bins, float* R_out, int32_t* best_out,
                                  float* best_R_out, void* hip_stream) {
    if (n_a < 0 || n_b < 0) return fail(SI_E_INVALID, "n_a and n_b must be >= 0");
    if (n_bins < 2 || n_bins > 65536) return fail(SI_E_INVALID, "n_bins must be in [2, 65536]");
    if (n_a >= INT32_MAX || n_b >= INT32_MAX)
        return fail(SI_E_INVALID, "n_a and n_b must be below 2^31 - 1");
    if (n_a == 0 || n_b == 0) return SI_OK;
    if (!A || !B) return fail(SI_E_INVALID, "A and B must be non-NULL");
    if (!R_out && !best_out && !best_R_out)
        return fail(SI_E_INVALID, "give at least one of R_out, best_out, best_R_out");
    hipStream_t s = (hipStream_t)hip_stream;
    const int Kp = (n_bins + kBK - 1) / kBK * kBK;
    const bool want_best = best_out || best_R_out;
    // one set against itself: its fp16 rows and sums serve as both operands
    const bool same = A == B && n_a == n_b;
    const size_t b_ha = rup256(sizeof(_Float16) * (size_t)n_a * Kp);
    const size_t b_hb = same ? 0 : rup256(sizeof(_Float16) * (size_t)n_b * Kp);
    const size_t b_sa = rup256(sizeof(float2) * (size_t)n_a);
    const size_t b_sb = same ? 0 : rup256(sizeof(float2) * (size_t)n_b);
    const size_t b_best = want_best ? rup256(sizeof(unsigned long long) * (size_t)n_a) : 0;
    char* m = nullptr;
    SI_HIP(pool_alloc((void**)&m, b_ha + b_hb + b_sa + b_sb + b_best, s));
    _Float16* HA = reinterpret_cast<_Float16*>(m);
    _Float16* HB = same ? HA : reinterpret_cast<_Float16*>(m + b_ha);
    float2* SA = reinterpret_cast<float2*>(m + b_ha + b_hb);
    float2* SB = same ? SA : reinterpret_cast<float2*>(m + b_ha + b_hb + b_sa);
    unsigned long long* best =
        want_best ? reinterpret_cast<unsigned long long*>(m + b_ha + b_hb + b_sa + b_sb) : nullptr;
    hipError_t e = hipSuccess;
    if (best) e = launch_fill(reinterpret_cast<int32_t*>(best), 2 * n_a, 0, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_corr_prep, dim3((unsigned)((n_a + 3) / 4)), dim3(256), 0, s, A, n_a,
                           (int)n_bins, Kp, HA, SA);
        if (!same)
            hipLaunchKernelGGL(k_corr_prep, dim3((unsigned)((n_b + 3) / 4)), dim3(256), 0, s, B,
                               n_b, (int)n_bins, Kp, HB, SB);
        const int64_t tiles_m = (n_a + kTM - 1) / kTM, tiles_n = (n_b + kTN - 1) / kTN;
        const int64_t super_m = (tiles_m + kSuperM - 1) / kSuperM;
        const int64_t super_n = (tiles_n + kSuperN - 1) / kSuperN;
        // every super-tile takes 64 workgroups, numbered 8 apart (one XCD)
        const int64_t grid = (super_m * super_n + 7) / 8 * 8 * (kSuperM * kSuperN);
        if (grid > INT32_MAX) e = hipErrorInvalidValue;
        else
            hipLaunchKernelGGL(k_corr_gemm, dim3((unsigned)grid), dim3(kGemmThreads), 0, s, HA,
                               HB, SA, SB, n_a, n_b, (int)n_bins, Kp, tiles_m, tiles_n, super_n,
                               R_out, best);
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e == hipSuccess && best) {
        hipLaunchKernelGGL(k_corr_best, dim3((unsigned)((n_a + 255) / 256)), dim3(256), 0, s, best,
                           n_a, best_out, best_R_out);
        e = hipGetLastError();
    }
    (void)hipFreeAsync(m, s);
    if (e != hipSuccess) return hip_fail(e, "spin-image correlation");
    return SI_OK;
}

extern "C" si_status si_estimate_normals(const float* points_xyz, int64_t M, float radius,
                                         const float* viewpoint, float* normals_out,
                                         int32_t* counts_out, void* hip_stream) {
    if (!points_xyz || !normals_out) return fail(SI_E_INVALID, "points or normals_out is NULL");
    if (!viewpoint) return fail(SI_E_INVALID, "viewpoint is NULL");
    if (M <= 0 || M >= INT32_MAX) return fail(SI_E_INVALID, "M must be in [1, 2^31 - 1)");
    if (!isfinite(radius) || !(radius > 0.0f)) return fail(SI_E_INVALID, "radius must be > 0");
    for (int k = 0; k < 3; ++k)
        if (!isfinite(viewpoint[k])) return fail(SI_E_INVALID, "viewpoint must be finite");
    // a grid whose cell edge is at least r (the scene's grid for a support
    // radius of 3r); the points stand in for the normals it does not read
    si_scene* sc = nullptr;
    si_status rc = si_build_scene(points_xyz, points_xyz, M, 3.0f * radius, hip_stream, &sc);
    if (rc != SI_OK) return rc;
    if (sc->h < (double)radius) {
        si_free_scene(sc);
        return fail(SI_E_DEVICE, "normal estimation: grid cell below the radius");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_normals, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, view_of(*sc),
                       radius, viewpoint[0], viewpoint[1], viewpoint[2], normals_out, counts_out);
    hipError_t e = hipGetLastError();
    si_free_scene(sc);  // waits for the kernel
    if (e != hipSuccess) return hip_fail(e, "normal estimation");
    return SI_OK;
}
