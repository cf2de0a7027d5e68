// Learned per-image cost model and the learned schedule.
//
// The earlier PSIA balanced CPU and co-processor work statically from per-image
// timings measured on each architecture (Section 2.3); here a small network
// predicts each image's cost from the occupancy of the grid around its
// oriented point, and the schedule orders and sizes chunks by the prediction:
//
//   features (12 per image) -> MLP 12-64-64-1 (ReLU, float32) -> log1p(count)
//   units of kUnit consecutive iterations of the cell-ordered loop, costed by
//   the sum of their predicted counts (+1 per image), taken in descending
//   cost (longest-processing-time first; a stable counting sort on a
//   logarithmic key), cut into chunks by factoring on predicted cost: batch b
//   has P chunks of ceil(R_b / (x P)) predicted cost each, R_b the cost left.
//
// Everything runs on the device, in the caller's stream.  Training uses
// hand-written forward/backward kernels whose reductions have a fixed order
// (per-block partial gradients, then a fixed-order sum over blocks), so a
// training run is reproducible, and Adam.  With no model the schedule falls
// back to FAC.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "si_internal.h"

struct si_cost_model {
    uint64_t serial = si::next_serial();
    int device = 0;
    uint64_t seed = 0;
    int64_t step = 0;        // Adam steps taken
    float* params = nullptr; // device, kNP
    float* m = nullptr;      // Adam first moment (device)
    float* v = nullptr;      // Adam second moment (device)
};

namespace si {

namespace {

constexpr int kNF = 12;                  // features
constexpr int kH = 64;                   // hidden width
constexpr int kNP = kH * kNF + kH + kH * kH + kH + kH + 1;  // 5057
constexpr int oW1 = 0, oB1 = kH * kNF, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH;
constexpr int kGradSamples = 32;         // samples per gradient block (8 threads each)
constexpr int kUnit = 16;                // iterations per learned-schedule unit
constexpr int kKeys = 1024;              // LPT key buckets (32 per octave of cost)
constexpr int kTile = 256;               // units per sort tile

// ---------------------------------------------------------------- features --
// Summed-volume table of a grid's cell counts: S(z, y, x) = points in the
// cells with cz < z, cy < y, cx < x, for 0 <= z <= dz, 0 <= y <= dy,
// 0 <= x <= dx, at ((z (dy + 1) + y) (dx + 1) + x).  Three passes: the
// counts along x come straight from the scene's key starts (a prefix along
// each row), then running sums along y and along z.
__host__ __device__ inline int64_t sat_entries(const int32_t* dims) {
    return (int64_t)(dims[0] + 1) * (dims[1] + 1) * (dims[2] + 1);
}

__device__ void sat_x_entry(const SceneView& sc, int32_t* S, int64_t e) {
    const int64_t X = sc.dims[0] + 1, Y = sc.dims[1] + 1;
    const int x = (int)(e % X);
    const int64_t t = e / X;
    const int y = (int)(t % Y), z = (int)(t / Y);
    int32_t v = 0;
    if (y > 0 && z > 0) {
        const int64_t row = ((int64_t)(z - 1) * sc.dims[1] + (y - 1)) * sc.dims[0];
        v = sc.sub_start[(row + x) * kSubX] - sc.sub_start[row * kSubX];
    }
    S[e] = v;
}

// Running sum of len entries base, base + stride, ... (eight loads in flight).
__device__ void sat_column(int32_t* S, int64_t base, int64_t stride, int len) {
    int32_t run = 0;
    int k = 0;
    for (; k + 8 <= len; k += 8) {
        int32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = S[base + (k + j) * stride];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            run += v[j];
            S[base + (k + j) * stride] = run;
        }
    }
    for (; k < len; ++k) {
        run += S[base + k * stride];
        S[base + k * stride] = run;
    }
}

// axis 0: pass along x (entries); 1: running sums along y (columns z, x);
// 2: along z (columns y, x)
__device__ void sat_step(const SceneView& sc, int32_t* S, int axis, int64_t t) {
    const int64_t X = sc.dims[0] + 1, Y = sc.dims[1] + 1, Z = sc.dims[2] + 1;
    if (axis == 0) {
        sat_x_entry(sc, S, t);
    } else if (axis == 1) {
        sat_column(S, (t / X) * Y * X + t % X, X, (int)Y);
    } else {
        sat_column(S, t, X * Y, (int)Z);
    }
}

__global__ void __launch_bounds__(256) k_sat(SceneView sc, int32_t* __restrict__ S, int axis,
                                             int64_t n) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) sat_step(sc, S, axis, t);
}

// Largest i < n with off[i] <= t (off ascending, off[0] <= t).
__device__ __forceinline__ int find_off(const int64_t* off, int n, int64_t t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The same for element t = blockIdx.x * blockDim.x + threadIdx.x: the search
// for the block's first element is the same in every lane (uniform loads),
// then each thread steps over the few offsets inside the block.
__device__ __forceinline__ int find_off_block(const int64_t* off, int n, int64_t t) {
    int i = find_off(off, n, (int64_t)blockIdx.x * blockDim.x);
    while (i + 1 < n && off[i + 1] <= t) ++i;
    return i;
}

// The same over the items of a batch: off holds 3 (n_items + 1) prefix
// offsets (entries, y columns, z columns); item i's table starts at entry
// off[i].
__global__ void __launch_bounds__(256) k_sat_multi(const Item* __restrict__ items, int n_items,
                                                   const int64_t* __restrict__ off,
                                                   int32_t* __restrict__ S, int axis) {
    const int64_t* o = off + (size_t)axis * (n_items + 1);
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= o[n_items]) return;
    const int i = find_off_block(o, n_items, t);
    sat_step(items[i].scene, S + off[i], axis, t - o[i]);
}

hipError_t launch_sat(const SceneView& sc, int32_t* S, hipStream_t s) {
    const int64_t X = sc.dims[0] + 1, Y = sc.dims[1] + 1, Z = sc.dims[2] + 1;
    const int64_t n[3] = {X * Y * Z, X * Z, X * Y};
    for (int axis = 0; axis < 3; ++axis)
        hipLaunchKernelGGL(k_sat, dim3((unsigned)((n[axis] + 255) / 256)), dim3(256), 0, s, sc, S,
                           axis, n[axis]);
    return hipGetLastError();
}

// The 12 features of oriented point o of the scene into f: from S, the
// scene's summed-volume table (TABLE), or by summing the block's grid rows
// directly (the same integer counts).
template <bool TABLE>
__device__ void features_of(const SceneView& sc, const int32_t* S, int o, float f11, float* f) {
    if (o < 0 || o >= sc.M) {
        for (int k = 0; k < kNF; ++k) f[k] = 0.0f;
        return;
    }
    const int sp = sc.inv[o];
    const float4 pa = sc.pos[sp];
    const float4 na = sc.nrm[sp];
    const int cell = __float_as_int(pa.w);
    const int c[3] = {cell % sc.dims[0], (cell / sc.dims[0]) % sc.dims[1],
                      cell / (sc.dims[0] * sc.dims[1])};
    const int half = kSub / 2;
    // point counts of the 3 x 3 x 3 coarse cells around p: coarse offset d
    // covers fine cells c + kSub d - half .. c + kSub d + half on each axis
    // (clipped to the grid), from the table at the 4 x 4 x 4 coarse corners
    int bnd[3][4];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int e[4] = {c[a] - kSub - half, c[a] - half, c[a] + half + 1, c[a] + kSub + half + 1};
#pragma unroll
        for (int b = 0; b < 4; ++b) bnd[a][b] = min(max(e[b], 0), sc.dims[a]);
    }
    int occ[3][3][3] = {};
    if (TABLE) {
        const int64_t X = sc.dims[0] + 1, Y = sc.dims[1] + 1;
        int V[4][4][4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    V[k][j][i] = S[((int64_t)bnd[2][k] * Y + bnd[1][j]) * X + bnd[0][i]];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
                    occ[dz][dy][dx] = V[dz + 1][dy + 1][dx + 1] - V[dz][dy + 1][dx + 1] -
                                      V[dz + 1][dy][dx + 1] - V[dz + 1][dy + 1][dx] +
                                      V[dz][dy][dx + 1] + V[dz][dy + 1][dx] +
                                      V[dz + 1][dy][dx] - V[dz][dy][dx];
    } else {
        // without a table: each fine row (y, z) of the block adds its counts
        // between the four x boundaries (every kSubX-th entry of sub_start)
        for (int z = bnd[2][0]; z < bnd[2][3]; ++z) {
            const int dz = z < bnd[2][1] ? 0 : (z < bnd[2][2] ? 1 : 2);
            for (int y = bnd[1][0]; y < bnd[1][3]; ++y) {
                const int dy = y < bnd[1][1] ? 0 : (y < bnd[1][2] ? 1 : 2);
                const int64_t row = ((int64_t)z * sc.dims[1] + y) * sc.dims[0];
                int e[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) e[b] = sc.sub_start[(row + bnd[0][b]) * kSubX];
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) occ[dz][dy][dx] += e[dx + 1] - e[dx];
            }
        }
    }
    float shell[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float tot = 0.0f, mx = 0.0f, my = 0.0f, mz = 0.0f, s8 = 0.0f, s9 = 0.0f;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const float o_ = (float)occ[dz + 1][dy + 1][dx + 1];
                shell[abs(dx) + abs(dy) + abs(dz)] += o_;
                tot += o_;
                mx += o_ * dx;
                my += o_ * dy;
                mz += o_ * dz;
                const float dn = dx * na.x + dy * na.y + dz * na.z;
                s8 += o_ * dn * dn;
                const float ex = dx - dn * na.x, ey = dy - dn * na.y, ez = dz - dn * na.z;
                s9 += o_ * (ex * ex + ey * ey + ez * ez);
            }
        }
    }
    const float inv = tot > 0.0f ? 1.0f / tot : 0.0f;
    for (int k = 0; k < 4; ++k) f[k] = log1pf(shell[k]);
    f[4] = mx * inv;
    f[5] = my * inv;
    f[6] = mz * inv;
    f[7] = f[4] * na.x + f[5] * na.y + f[6] * na.z;
    f[8] = s8 * inv;
    f[9] = s9 * inv;
    f[10] = log1pf(tot);
    f[11] = f11;
}

template <bool TABLE>
__global__ void __launch_bounds__(256) k_features(SceneView sc, const int32_t* __restrict__ S,
                                                  const int32_t* __restrict__ oriented,
                                                  int64_t N, float f11, float* __restrict__ feats) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    features_of<TABLE>(sc, S, oriented[i], f11, feats + kNF * i);
}

// Features of loop position t (iteration perm[t], or t) into feats[t]: in the
// cell order, the lanes of a wave read the same grid rows.
template <bool TABLE>
__global__ void __launch_bounds__(256) k_features_loop(SceneView sc,
                                                       const int32_t* __restrict__ S,
                                                       const int32_t* __restrict__ oriented,
                                                       const int32_t* __restrict__ perm,
                                                       int64_t N, float f11,
                                                       float* __restrict__ feats) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N) return;
    features_of<TABLE>(sc, S, oriented[perm ? perm[t] : t], f11, feats + kNF * t);
}

// ------------------------------------------------------------- MLP forward --
// pred[i] = max(expm1(net(feats[i])), 0); with `out_raw` the raw network
// output is written instead.
__global__ void __launch_bounds__(256) k_mlp_predict(const float* __restrict__ params,
                                                     const float* __restrict__ feats, int64_t n,
                                                     float* __restrict__ pred, int out_raw) {
    __shared__ float P[kNP];
    for (int k = threadIdx.x; k < kNP; k += blockDim.x) P[k] = params[k];
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[kNF];
    for (int k = 0; k < kNF; ++k) x[k] = feats[kNF * i + k];
    float h1[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float z = P[oB1 + j];
#pragma unroll
        for (int k = 0; k < kNF; ++k) z = fmaf(P[oW1 + j * kNF + k], x[k], z);
        h1[j] = fmaxf(z, 0.0f);
    }
    float out = P[oB3];
    for (int j = 0; j < kH; ++j) {
        float z = P[oB2 + j];
#pragma unroll
        for (int k = 0; k < kH; ++k) z = fmaf(P[oW2 + j * kH + k], h1[k], z);
        out = fmaf(P[oW3 + j], fmaxf(z, 0.0f), out);
    }
    pred[i] = out_raw ? out : fmaxf(expm1f(out), 0.0f);
}

// -------------------------------------------- MLP forward on matrix cores --
// The learned schedule's planner evaluates the network with fp16 operands and
// fp32 accumulation on MFMA (v_mfma_f32_16x16x16_f16): per wave, 16 images at
// a time, products taken transposed (weights x activations) so that each
// layer's 16 x 16 output tiles are already the next layer's operand tiles:
//   H1^T = relu(W1 X^T + b1)    4 MFMA (neuron tiles t, K = 12 padded to 16)
//   H2^T = relu(W2 H1^T + b2)   16 MFMA (neuron tiles u, K steps s)
//   out  = w3 . H2^T + b3       per-lane dot products and two lane swaps
// Operand layout of the 16x16x16 product (wave of 64): lane l holds row
// l % 16 of A and column l % 16 of B at K = 4 (l / 16) .. + 3; the 16 x 16
// result has column l % 16, rows 4 (l / 16) .. + 3 in lane l.  Only the
// planner uses this path: the ordering it feeds groups costs 32 buckets per
// octave, far coarser than the fp16 rounding.
typedef _Float16 h16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4m __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_mlp_predict_mfma(const float* __restrict__ params,
                                                          const float* __restrict__ feats,
                                                          int64_t n, float* __restrict__ pred,
                                                          int out_raw) {
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, kb = lane >> 4;  // row/column within a tile, K block
    // weights as A operands, biases and w3 at this lane's result rows
    h16x4 a1[4], a2[4][4];
    float b1[4][4], b2[4][4], w3[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * kb + i;
            a1[t][i] = (_Float16)(k < kNF ? params[oW1 + (16 * t + r16) * kNF + k] : 0.0f);
            b1[t][i] = params[oB1 + 16 * t + 4 * kb + i];
            b2[t][i] = params[oB2 + 16 * t + 4 * kb + i];
            w3[t][i] = params[oW3 + 16 * t + 4 * kb + i];
        }
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a2[t][s2][i] = (_Float16)params[oW2 + (16 * t + r16) * kH + 16 * s2 + 4 * kb + i];
    }
    const float b3 = params[oB3];
    const int64_t n_tiles = (n + 15) / 16;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    // features 4 kb .. 4 kb + 3 of this lane's image of a tile (one 16-byte
    // load; K block 3 is the zero padding), the next tile's fetched while the
    // current one is computed
    auto load_x = [&](int64_t tile) {
        f32x4m v = {0.0f, 0.0f, 0.0f, 0.0f};
        const int64_t img = tile * 16 + r16;
        if (tile < n_tiles && img < n && kb < kNF / 4)
            v = *reinterpret_cast<const f32x4m*>(feats + kNF * img + 4 * kb);
        return v;
    };
    f32x4m xn = load_x(wave);
    for (int64_t tile = wave; tile < n_tiles; tile += n_waves) {
        const int64_t img = tile * 16 + r16;
        const f32x4m xf = xn;
        xn = load_x(tile + n_waves);
        // B operand of layer 1
        h16x4 x;
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = (_Float16)xf[i];
        h16x4 h1[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4m d = {0.0f, 0.0f, 0.0f, 0.0f};
            d = __builtin_amdgcn_mfma_f32_16x16x16f16(a1[t], x, d, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) h1[t][i] = (_Float16)fmaxf(d[i] + b1[t][i], 0.0f);
        }
        float part = 0.0f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            f32x4m d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2)
                d = __builtin_amdgcn_mfma_f32_16x16x16f16(a2[u][s2], h1[s2], d, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) part = fmaf(w3[u][i], fmaxf(d[i] + b2[u][i], 0.0f), part);
        }
        // the four lanes of image r16 hold the four quarters of the dot product
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        if (kb == 0 && img < n) {
            const float out = part + b3;
            pred[img] = out_raw ? out : fmaxf(expm1f(out), 0.0f);
        }
    }
}

hipError_t launch_mlp_predict_mfma(const float* params, const float* feats, int64_t n,
                                   float* pred, int out_raw, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    // every wave loads the weights once: about 32 tiles of 16 images per wave
    const int64_t tiles = (n + 15) / 16;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + 127) / 128, 1024));
    hipLaunchKernelGGL(k_mlp_predict_mfma, dim3(blocks), dim3(256), 0, s, params, feats, n, pred,
                       out_raw);
    return hipGetLastError();
}

// ---------------------------------------------------------------- gradient --
// One block: kGradSamples samples (8 threads each).  Samples are
// sel[start + s] (or start + s without sel), s < count.  Writes this block's
// gradient of sum_s (out_s - y_s)^2 * scale, and the block's summed squared
// error in slot kNP, to partial[blockIdx.x * (kNP + 1) ...].
__global__ void __launch_bounds__(256) k_mlp_grad(const float* __restrict__ params,
                                                  const float* __restrict__ feats,
                                                  const uint32_t* __restrict__ counts,
                                                  const int32_t* __restrict__ sel, int64_t start,
                                                  int64_t count, float scale,
                                                  float* __restrict__ partial) {
    __shared__ float X[kGradSamples][kNF];
    __shared__ float H1[kGradSamples][kH];
    __shared__ float H2[kGradSamples][kH];
    __shared__ float D2[kGradSamples][kH];
    __shared__ float D1[kGradSamples][kH];
    __shared__ float Dout[kGradSamples];
    __shared__ float Loss[kGradSamples];
    const int tid = threadIdx.x;
    const int s = tid >> 3, q = tid & 7;
    const int64_t b0 = start + (int64_t)blockIdx.x * kGradSamples;
    const int64_t my = b0 + s;
    const bool valid = (my - start) < count;
    int64_t row = 0;
    if (valid) row = sel ? sel[my] : my;
    for (int k = q; k < kNF; k += 8) X[s][k] = valid ? feats[kNF * row + k] : 0.0f;
    __syncthreads();
    for (int jj = 0; jj < 8; ++jj) {
        const int j = q * 8 + jj;
        float z = params[oB1 + j];
        for (int k = 0; k < kNF; ++k) z = fmaf(params[oW1 + j * kNF + k], X[s][k], z);
        H1[s][j] = fmaxf(z, 0.0f);
    }
    __syncthreads();
    for (int jj = 0; jj < 8; ++jj) {
        const int j = q * 8 + jj;
        float z = params[oB2 + j];
        for (int k = 0; k < kH; ++k) z = fmaf(params[oW2 + j * kH + k], H1[s][k], z);
        H2[s][j] = fmaxf(z, 0.0f);
    }
    __syncthreads();
    if (q == 0) {
        float out = params[oB3];
        for (int j = 0; j < kH; ++j) out = fmaf(params[oW3 + j], H2[s][j], out);
        const float y = valid ? log1pf((float)counts[row]) : 0.0f;
        const float r = out - y;
        Dout[s] = valid ? 2.0f * r * scale : 0.0f;
        Loss[s] = valid ? r * r : 0.0f;
    }
    __syncthreads();
    for (int jj = 0; jj < 8; ++jj) {
        const int j = q * 8 + jj;
        D2[s][j] = H2[s][j] > 0.0f ? Dout[s] * params[oW3 + j] : 0.0f;
    }
    __syncthreads();
    for (int kk = 0; kk < 8; ++kk) {
        const int k = q * 8 + kk;
        float g = 0.0f;
        for (int j = 0; j < kH; ++j) g = fmaf(params[oW2 + j * kH + k], D2[s][j], g);
        D1[s][k] = H1[s][k] > 0.0f ? g : 0.0f;
    }
    __syncthreads();
    float* out = partial + (size_t)blockIdx.x * (kNP + 1);
    for (int p = tid; p < kNP; p += blockDim.x) {
        float g = 0.0f;
        if (p < oB1) {
            const int j = p / kNF, i = p % kNF;
            for (int t = 0; t < kGradSamples; ++t) g = fmaf(D1[t][j], X[t][i], g);
        } else if (p < oW2) {
            const int j = p - oB1;
            for (int t = 0; t < kGradSamples; ++t) g += D1[t][j];
        } else if (p < oB2) {
            const int r = p - oW2, j = r / kH, k = r % kH;
            for (int t = 0; t < kGradSamples; ++t) g = fmaf(D2[t][j], H1[t][k], g);
        } else if (p < oW3) {
            const int j = p - oB2;
            for (int t = 0; t < kGradSamples; ++t) g += D2[t][j];
        } else if (p < oB3) {
            const int j = p - oW3;
            for (int t = 0; t < kGradSamples; ++t) g = fmaf(Dout[t], H2[t][j], g);
        } else {
            for (int t = 0; t < kGradSamples; ++t) g += Dout[t];
        }
        out[p] = g;
    }
    if (tid == 0) {
        float l = 0.0f;
        for (int t = 0; t < kGradSamples; ++t) l += Loss[t];
        out[kNP] = l;
    }
}

// grad[p] = sum over blocks (fixed order); loss_acc[0] += summed loss.
__global__ void __launch_bounds__(256) k_mlp_reduce(const float* __restrict__ partial, int nblk,
                                                    float* __restrict__ grad,
                                                    float* __restrict__ loss_acc) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNP) return;
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += partial[(size_t)b * (kNP + 1) + p];
    if (p < kNP) grad[p] = g;
    else if (loss_acc) loss_acc[0] += g;
}

__global__ void __launch_bounds__(256) k_adam(float* __restrict__ params, const float* __restrict__ grad,
                                              float* __restrict__ m, float* __restrict__ v, float lr,
                                              float bc1, float bc2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNP) return;
    const float g = grad[p];
    const float mm = 0.9f * m[p] + 0.1f * g;
    const float vv = 0.999f * v[p] + 0.001f * g * g;
    m[p] = mm;
    v[p] = vv;
    params[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
}

// ------------------------------------------------------- learned schedule --
// Unit u covers iterations [u*kUnit, min(N, (u+1)*kUnit)) of the work order;
// its integer cost is round(sum over its images of (pred + 1)); its key puts
// larger costs first.
__global__ void __launch_bounds__(256) k_unit_cost(const float* __restrict__ pred,
                                                   const int32_t* __restrict__ perm0, int64_t N,
                                                   int64_t n_units, uint32_t* __restrict__ qcost,
                                                   int32_t* __restrict__ key) {
    const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (u >= n_units) return;
    const int64_t a = u * kUnit, b = min((int64_t)N, a + kUnit);
    float c = 0.0f;
    for (int64_t t = a; t < b; ++t) {
        const float pv = pred[perm0 ? perm0[t] : t];
        c += (pv == pv) ? fminf(pv, 1e7f) + 1.0f : 1.0f;  // a non-finite prediction costs 1
    }
    const uint32_t q = (uint32_t)fmaxf(rintf(c), 1.0f);
    qcost[u] = q;
    const int k = (int)floorf(log2f((float)q) * 32.0f);
    key[u] = kKeys - 1 - min(max(k, 0), kKeys - 1);
}

// Per tile of kTile units: key histogram and each unit's rank among the
// earlier units of its tile with the same key (a stable order).
__global__ void __launch_bounds__(kTile) k_unit_hist(const int32_t* __restrict__ key, int64_t n_units,
                                                     int32_t* __restrict__ tile_hist,
                                                     int32_t* __restrict__ rank) {
    __shared__ int hist[kKeys];
    __shared__ int keys[kTile];
    for (int k = threadIdx.x; k < kKeys; k += kTile) hist[k] = 0;
    const int64_t u = (int64_t)blockIdx.x * kTile + threadIdx.x;
    const int my = u < n_units ? key[u] : -1;
    keys[threadIdx.x] = my;
    __syncthreads();
    if (my >= 0) {
        atomicAdd(&hist[my], 1);
        int r = 0;
        for (int t = 0; t < (int)threadIdx.x; ++t) r += keys[t] == my;
        rank[u] = r;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kKeys; k += kTile)
        tile_hist[(size_t)blockIdx.x * kKeys + k] = hist[k];
}

// Exclusive offsets of key k over the tiles (block k): tile_hist[t][k] <- units
// of key k in tiles < t; key_total[k] <- units of key k.
__global__ void __launch_bounds__(256) k_unit_tile_scan(int32_t* __restrict__ tile_hist, int n_tiles,
                                                        int32_t* __restrict__ key_total) {
    __shared__ int sc[256];
    __shared__ int carry;
    const int k = blockIdx.x, tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int t0 = 0; t0 < n_tiles; t0 += 256) {
        const int t = t0 + tid;
        const int v = t < n_tiles ? tile_hist[(size_t)t * kKeys + k] : 0;
        sc[tid] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int a = tid >= off ? sc[tid - off] : 0;
            __syncthreads();
            sc[tid] += a;
            __syncthreads();
        }
        if (t < n_tiles) tile_hist[(size_t)t * kKeys + k] = carry + sc[tid] - v;
        __syncthreads();
        if (tid == 255) carry += sc[255];
        __syncthreads();
    }
    if (tid == 0) key_total[k] = carry;
}

// key_base[k] = units of all keys < k (one block of kKeys threads).
__global__ void __launch_bounds__(kKeys) k_unit_key_base(const int32_t* __restrict__ key_total,
                                                         int32_t* __restrict__ key_base) {
    __shared__ int sc[kKeys];
    const int k = threadIdx.x;
    const int v = key_total[k];
    sc[k] = v;
    __syncthreads();
    for (int off = 1; off < kKeys; off <<= 1) {
        const int a = k >= off ? sc[k - off] : 0;
        __syncthreads();
        sc[k] += a;
        __syncthreads();
    }
    key_base[k] = sc[k] - v;
}

__global__ void __launch_bounds__(256) k_unit_scatter(const int32_t* __restrict__ key,
                                                      const int32_t* __restrict__ rank,
                                                      const int32_t* __restrict__ tile_hist,
                                                      const int32_t* __restrict__ key_base,
                                                      int64_t n_units, int32_t* __restrict__ order) {
    const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (u >= n_units) return;
    const int64_t t = u / kTile;
    const int k = key[u];
    order[key_base[k] + tile_hist[t * kKeys + k] + rank[u]] = (int32_t)u;
}

// Per LPT position k: the cost and the iteration count of unit order[k].
__global__ void __launch_bounds__(256) k_unit_gather(const int32_t* __restrict__ order,
                                                     const uint32_t* __restrict__ qcost,
                                                     int64_t n_units, int64_t N,
                                                     int64_t* __restrict__ cval,
                                                     int64_t* __restrict__ ival) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n_units) return;
    const int64_t u = order[k];
    cval[k] = qcost[u];
    ival[k] = min((int64_t)kUnit, N - u * kUnit);
}

// Search structure for factoring on cost: the exclusive cost prefix cpre
// (nondecreasing, n + 1 entries) sampled every `stride` entries into LDS, so
// that finding the first entry >= a target takes a binary search in LDS and
// one over a window of `stride` entries in global memory.
constexpr int kCostSamples = 4096;
struct CostIndex {
    const int64_t* cpre;
    int64_t n;
    int64_t stride;
    int ns;          // samples: entry min(i * stride, n) for i < ns
    int64_t* samp;   // LDS, ns values
};

// Fill the index (all threads of the block; a barrier follows).
__device__ CostIndex cost_index(const int64_t* cpre, int64_t n, int64_t* samp) {
    CostIndex ix;
    ix.cpre = cpre;
    ix.n = n;
    ix.stride = max((int64_t)1, (n + kCostSamples - 2) / (kCostSamples - 1));
    ix.ns = (int)((n + ix.stride - 1) / ix.stride) + 1;
    ix.samp = samp;
    for (int i = threadIdx.x; i < ix.ns; i += blockDim.x)
        samp[i] = cpre[min((int64_t)i * ix.stride, n)];
    __syncthreads();
    return ix;
}

// First k in [0, n] with cpre[k] >= target, or n + 1 if there is none.
__device__ int64_t first_at_least(const CostIndex& ix, int64_t target) {
    if (ix.samp[0] >= target) return 0;
    int lo = 0, hi = ix.ns - 1;  // largest sample below the target
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ix.samp[mid] < target) lo = mid; else hi = mid - 1;
    }
    if (lo == ix.ns - 1) return ix.n + 1;
    int64_t a = (int64_t)lo * ix.stride + 1;
    int64_t b = min((int64_t)(lo + 1) * ix.stride, ix.n);  // cpre[b] >= target
    while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (ix.cpre[mid] >= target) b = mid; else a = mid + 1;
    }
    return a;
}

// End of chunk j of the batch starting at st with chunk cost cb: the first
// k in [st + 1, n) with cpre[k] - cpre[st] >= j * cb, else n.
__device__ __forceinline__ int64_t chunk_end(const CostIndex& ix, int64_t st, int64_t c_st,
                                             int64_t j, int64_t cb) {
    return min(ix.n, max(st + 1, first_at_least(ix, c_st + j * cb)));
}

// Single block: factoring on predicted cost over the LPT order (cpre, ipre:
// exclusive prefix sums of cost and iterations, n_units + 1 entries), the
// chunk table and its length.  Thread t computes chunks t*kPerThread+1 ..
// (t+1)*kPerThread of each batch of P <= kMaxLearnedP.
constexpr int kPerThread = kMaxLearnedP / 1024;
__global__ void __launch_bounds__(1024) k_learned_chunks(const int64_t* __restrict__ cpre,
                                                         const int64_t* __restrict__ ipre,
                                                         int64_t n_units, int P, float divisor,
                                                         Chunk* __restrict__ chunks,
                                                         int32_t* __restrict__ n_chunks) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t total = cpre[n_units];
    __shared__ int64_t start;
    __shared__ int emitted;
    __shared__ int32_t ends[kMaxLearnedP + 1];
    __shared__ int wsum[1024 / 64];
    __shared__ int64_t samp[kCostSamples];
    if (tid == 0) {
        start = 0;
        emitted = 0;
    }
    const CostIndex ix = cost_index(cpre, n_units, samp);
    const double x = divisor > 0.0f ? (double)divisor : 2.0;
    while (start < n_units) {
        const int64_t st = start;
        const int64_t c_st = cpre[st];
        const int64_t R = total - c_st;
        const int64_t cb = max((int64_t)1, (int64_t)ceil((double)R / (x * (double)P)));
        // end of chunk j (1..P): first k > st with cpre[k] - cpre[st] >= j * cb,
        // else n_units (every thread takes every 1024th j: independent searches)
        for (int j = tid + 1; j <= P; j += 1024) ends[j] = (int32_t)chunk_end(ix, st, c_st, j, cb);
        if (tid == 0) ends[0] = (int32_t)st;
        __syncthreads();
        // non-empty chunks of the batch, written in order (block prefix sum
        // over runs of kPerThread consecutive j)
        int mine = 0;
        for (int r = 0; r < kPerThread; ++r) {
            const int j = tid * kPerThread + r + 1;
            if (j <= P && ends[j] > ends[j - 1]) ++mine;
        }
        // block scan: shuffles inside each wave, then the 16 wave totals
        int incl = mine;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int before = 0, all = 0;
        for (int q = 0; q < 1024 / 64; ++q) {
            const int t = wsum[q];
            before += q < wave ? t : 0;
            all += t;
        }
        int w = emitted + before + incl - mine;
        for (int r = 0; r < kPerThread; ++r) {
            const int j = tid * kPerThread + r + 1;
            if (j <= P && ends[j] > ends[j - 1]) {
                Chunk c;
                c.item = 0;
                c.start = (int32_t)ipre[ends[j - 1]];
                c.end = (int32_t)ipre[ends[j]];
                chunks[w++] = c;
            }
        }
        __syncthreads();
        if (tid == 0) {
            emitted += all;
            start = ends[P];
        }
        __syncthreads();
    }
    if (tid == 0) *n_chunks = emitted;
}

// Iteration -> output position of the learned order.
__global__ void __launch_bounds__(256) k_learned_perm(const int32_t* __restrict__ order,
                                                      const int64_t* __restrict__ ipre,
                                                      const int32_t* __restrict__ perm0,
                                                      int64_t N, int64_t n_units,
                                                      int32_t* __restrict__ perm) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n_units) return;
    const int64_t u = order[k];
    const int64_t a = u * kUnit, len = min((int64_t)kUnit, N - a);
    const int64_t o = ipre[k];
    for (int64_t r = 0; r < len; ++r) perm[o + r] = perm0 ? perm0[a + r] : (int32_t)(a + r);
}

// ------------------------------------------ learned schedule, many items --
// The loop of a batched launch is the concatenation of the items' loops
// (cell-ordered within each item).  Units never cross an item: item i has
// units unit_off[i] .. unit_off[i+1]-1 of kUnit iterations (the last one
// shorter).  All units are put in one LPT order (stable by cost key, so
// within a key by item, then by unit) and cut by factoring on predicted cost
// into global chunks; a global chunk is split into its runs of one item.
// Item i's units, taken in LPT order, are its new loop order, so every run is
// a contiguous range of that order: the segment of (key k, item i) starts at
// base_len[i][k] = iterations of item i's units with keys < k.

// Features of flattened iteration t (the image of item i's iteration
// perm_cell[t], or t - item_off[i] without a cell order).
template <bool TABLE>
__global__ void __launch_bounds__(256) k_features_multi(const Item* __restrict__ items,
                                                        const int64_t* __restrict__ item_off,
                                                        int n_items,
                                                        const int32_t* __restrict__ perm_cell,
                                                        const float* __restrict__ f11,
                                                        const int64_t* __restrict__ sat_off,
                                                        const int32_t* __restrict__ sat,
                                                        int64_t total_N, float* __restrict__ feats) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= total_N) return;
    const int i = find_off_block(item_off, n_items, t);
    const Item& it = items[i];
    const int w = perm_cell ? perm_cell[t] : (int)(t - item_off[i]);
    // items with a table have entries in it; the other launch takes the rest
    if ((sat_off[i + 1] > sat_off[i]) != TABLE) return;
    features_of<TABLE>(it.scene, sat + sat_off[i], it.oriented[w], f11[i], feats + kNF * t);
}

}  // namespace

// Summed-volume tables of the items' grids (sat_off: entry and column
// offsets as sat_offsets writes them), then the features of every loop
// position t of the concatenated items (item-local iteration perm_cell[t],
// or t - item_off[i]) into feats[t].
hipError_t launch_features_multi(const Item* items, const int64_t* item_off, int n_items,
                                 const int32_t* perm_cell, const float* f11,
                                 const int64_t* sat_off, int32_t* sat, const int64_t pass_n[3],
                                 int64_t total_N, float* feats, hipStream_t s) {
    // pass_n: entries, y columns and z columns over all items (host copies of
    // the last offsets)
    for (int axis = 0; axis < 3; ++axis)
        if (pass_n[axis] > 0)
            hipLaunchKernelGGL(k_sat_multi, dim3((unsigned)((pass_n[axis] + 255) / 256)), dim3(256),
                               0, s, items, n_items, sat_off, sat, axis);
    const dim3 grid((unsigned)((total_N + 255) / 256));
    if (pass_n[0] > 0)
        hipLaunchKernelGGL(k_features_multi<true>, grid, dim3(256), 0, s, items, item_off, n_items,
                           perm_cell, f11, sat_off, sat, total_N, feats);
    hipLaunchKernelGGL(k_features_multi<false>, grid, dim3(256), 0, s, items, item_off, n_items,
                       perm_cell, f11, sat_off, sat, total_N, feats);
    return hipGetLastError();
}

namespace {

// Cost and key of unit u (as k_unit_cost), its length and item, and the
// per-(item, key) unit and iteration counts.
__global__ void __launch_bounds__(256) k_unit_cost_multi(
    const float* __restrict__ pred, const int64_t* __restrict__ unit_off,
    const int64_t* __restrict__ item_off, int n_items, int64_t n_units,
    uint32_t* __restrict__ qcost, int32_t* __restrict__ key, int32_t* __restrict__ ulen,
    int32_t* __restrict__ uitem, int32_t* __restrict__ hcount, int32_t* __restrict__ hlen) {
    const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (u >= n_units) return;
    const int i = find_off_block(unit_off, n_items, u);
    const int64_t a = item_off[i] + (u - unit_off[i]) * kUnit;
    const int64_t b = min(item_off[i + 1], a + kUnit);
    float c = 0.0f;
    for (int64_t t = a; t < b; ++t) {
        const float pv = pred[t];
        c += (pv == pv) ? fminf(pv, 1e7f) + 1.0f : 1.0f;  // a non-finite prediction costs 1
    }
    const uint32_t q = (uint32_t)fmaxf(rintf(c), 1.0f);
    qcost[u] = q;
    const int k = kKeys - 1 - min(max((int)floorf(log2f((float)q) * 32.0f), 0), kKeys - 1);
    key[u] = k;
    ulen[u] = (int32_t)(b - a);
    uitem[u] = i;
    atomicAdd(hcount + (size_t)i * kKeys + k, 1);
    atomicAdd(hlen + (size_t)i * kKeys + k, (int32_t)(b - a));
}

__global__ void __launch_bounds__(256) k_unit_gather_multi(const int32_t* __restrict__ order,
                                                           const uint32_t* __restrict__ qcost,
                                                           const int32_t* __restrict__ ulen,
                                                           int64_t n_units,
                                                           int64_t* __restrict__ cval,
                                                           int64_t* __restrict__ ival) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n_units) return;
    const int64_t u = order[k];
    cval[k] = qcost[u];
    ival[k] = ulen[u];
}

// Single block: factoring on predicted cost over the LPT order (cpre:
// exclusive prefix of cost, n_units + 1 entries); marks the first LPT
// position of every non-empty global chunk in cut (zeroed by the caller).
// ends: P + 1 int64 of scratch.
__global__ void __launch_bounds__(1024) k_learned_cuts(const int64_t* __restrict__ cpre,
                                                       int64_t n_units, int P, float divisor,
                                                       int64_t* __restrict__ ends,
                                                       int32_t* __restrict__ cut) {
    const int tid = threadIdx.x;
    const int64_t total = cpre[n_units];
    __shared__ int64_t start;
    __shared__ int64_t samp[kCostSamples];
    if (tid == 0) start = 0;
    const CostIndex ix = cost_index(cpre, n_units, samp);
    const double x = divisor > 0.0f ? (double)divisor : 2.0;
    while (start < n_units) {
        const int64_t st = start;
        const int64_t c_st = cpre[st];
        const int64_t R = total - c_st;
        const int64_t cb = max((int64_t)1, (int64_t)ceil((double)R / (x * (double)P)));
        for (int j = tid + 1; j <= P; j += 1024) ends[j] = chunk_end(ix, st, c_st, j, cb);
        if (tid == 0) ends[0] = st;
        __syncthreads();
        for (int j = tid + 1; j <= P; j += 1024)
            if (ends[j] > ends[j - 1]) cut[ends[j - 1]] = 1;
        __syncthreads();
        if (tid == 0) start = ends[P];
        __syncthreads();
    }
}

// base_len[i][k] = iterations of item i's units with keys < k (block i).
__global__ void __launch_bounds__(kKeys) k_item_key_base(const int32_t* __restrict__ hlen,
                                                         int32_t* __restrict__ base_len) {
    __shared__ int sc[kKeys];
    const int k = threadIdx.x;
    const size_t row = (size_t)blockIdx.x * kKeys;
    const int v = hlen[row + k];
    sc[k] = v;
    __syncthreads();
    for (int off = 1; off < kKeys; off <<= 1) {
        const int a = k >= off ? sc[k - off] : 0;
        __syncthreads();
        sc[k] += a;
        __syncthreads();
    }
    base_len[row + k] = sc[k] - v;
}

// seg_first[k][i] = LPT position of the first unit of (key k, item i):
// key_base[k] + units of key k in items < i (block k).
__global__ void __launch_bounds__(256) k_seg_first(const int32_t* __restrict__ hcount,
                                                   const int32_t* __restrict__ key_base,
                                                   int n_items, int32_t* __restrict__ seg_first) {
    __shared__ int sc[256];
    __shared__ int carry;
    const int k = blockIdx.x, tid = threadIdx.x;
    if (tid == 0) carry = key_base[k];
    __syncthreads();
    for (int i0 = 0; i0 < n_items; i0 += 256) {
        const int i = i0 + tid;
        const int v = i < n_items ? hcount[(size_t)i * kKeys + k] : 0;
        sc[tid] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int a = tid >= off ? sc[tid - off] : 0;
            __syncthreads();
            sc[tid] += a;
            __syncthreads();
        }
        if (i < n_items) seg_first[(size_t)k * n_items + i] = carry + sc[tid] - v;
        __syncthreads();
        if (tid == 255) carry += sc[255];
        __syncthreads();
    }
}

// Per LPT position k: the unit's offset in its item's new order, its
// iterations written there, and whether a run (sub-chunk) starts at k.
__global__ void __launch_bounds__(256) k_learned_perm_multi(
    const int32_t* __restrict__ order, const int32_t* __restrict__ key,
    const int32_t* __restrict__ ulen, const int32_t* __restrict__ uitem,
    const int64_t* __restrict__ unit_off, const int64_t* __restrict__ item_off, int n_items,
    const int64_t* __restrict__ ipre, const int32_t* __restrict__ base_len,
    const int32_t* __restrict__ seg_first, const int32_t* __restrict__ cut,
    const int32_t* __restrict__ perm_cell, int64_t n_units, int32_t* __restrict__ offs,
    int32_t* __restrict__ flag, int32_t* __restrict__ perm) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n_units) return;
    const int64_t u = order[k];
    const int i = uitem[u];
    const int kk = key[u];
    const int64_t first = seg_first[(size_t)kk * n_items + i];
    const int32_t off = base_len[(size_t)i * kKeys + kk] + (int32_t)(ipre[k] - ipre[first]);
    offs[k] = off;
    flag[k] = (k == 0 || cut[k] || uitem[order[k - 1]] != i) ? 1 : 0;
    const int64_t a = item_off[i] + (u - unit_off[i]) * kUnit;
    const int len = ulen[u];
    int32_t* dst = perm + item_off[i] + off;
    for (int r = 0; r < len; ++r)
        dst[r] = perm_cell ? perm_cell[a + r] : (int32_t)(a + r - item_off[i]);
}

// Sub-chunks from the run starts: fpre = exclusive prefix of flag
// (n_units + 1 entries).
__global__ void __launch_bounds__(256) k_emit_runs(const int32_t* __restrict__ order,
                                                   const int32_t* __restrict__ uitem,
                                                   const int32_t* __restrict__ ulen,
                                                   const int32_t* __restrict__ offs,
                                                   const int32_t* __restrict__ flag,
                                                   const int32_t* __restrict__ fpre,
                                                   int64_t n_units, Chunk* __restrict__ chunks,
                                                   int32_t* __restrict__ n_chunks) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n_units) return;
    const int c = fpre[k + 1] - 1;  // run holding position k
    if (flag[k]) {
        chunks[c].item = uitem[order[k]];
        chunks[c].start = offs[k];
    }
    if (k == n_units - 1 || flag[k + 1]) chunks[c].end = offs[k] + ulen[order[k]];
    if (k == n_units - 1) *n_chunks = fpre[n_units];
}

uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t& s) { return (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

unsigned nblocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

si_status features_launch(const Scene& sc, const int32_t* oriented, int64_t N,
                          const si_params* params, float* feats, hipStream_t s) {
    SpinParams p;
    double R;
    si_status rc = make_params(params, &p, &R);
    if (rc != SI_OK) return rc;
    const float f11 = (float)(R / (kSub * sc.h));
    const SceneView v = view_of(sc);
    int32_t* S = nullptr;
    hipError_t e = hipSuccess;
    if (use_feature_table(v.dims, N)) {
        SI_HIP(pool_alloc((void**)&S, sizeof(int32_t) * sat_entries(v.dims), s));
        e = launch_sat(v, S, s);
    }
    if (e == hipSuccess) {
        if (S)
            hipLaunchKernelGGL(k_features<true>, dim3(nblocks(N)), dim3(256), 0, s, v, S, oriented,
                               N, f11, feats);
        else
            hipLaunchKernelGGL(k_features<false>, dim3(nblocks(N)), dim3(256), 0, s, v, S,
                               oriented, N, f11, feats);
        e = hipGetLastError();
    }
    if (S) (void)hipFreeAsync(S, s);
    if (e != hipSuccess) return hip_fail(e, "features");
    return SI_OK;
}

si_status learned_table(DeviceState*, const Scene* scene, const int32_t* oriented, int64_t N,
                        const si_params* params, const si_sched* sched, int n_wg, int,
                        LearnedPlan* plan, hipStream_t s) {
    const si_cost_model* model = sched->model;
    if (!model) return fail(SI_E_UNSUPPORTED, "learned schedule without a model");
    if (n_wg > kMaxLearnedP)
        return fail(SI_E_INVALID, "the learned schedule supports at most 4096 workgroups");
    const int64_t n_units = (N + kUnit - 1) / kUnit;
    const int64_t n_tiles = (n_units + kTile - 1) / kTile;
    const int64_t nt = scan_tmp_elems(scene->M);
    // one stream-ordered block for every temporary
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) & ~(size_t)255; return r; };
    const size_t o_perm0 = take(sizeof(int32_t) * N);
    const size_t o_key = take(sizeof(int32_t) * N);
    const size_t o_rank = take(sizeof(int32_t) * N);
    const size_t o_counts = take(sizeof(int32_t) * scene->M);
    const size_t o_starts = take(sizeof(int32_t) * (scene->M + 1));
    const size_t o_tmp = take(sizeof(int32_t) * nt);
    const size_t o_feats = take(sizeof(float) * kNF * N);
    const bool table = use_feature_table(scene->dims, N);
    const size_t o_sat = take(sizeof(int32_t) * (table ? sat_entries(scene->dims) : 1));
    const size_t o_pred = take(sizeof(float) * N);
    const size_t o_qcost = take(sizeof(uint32_t) * n_units);
    const size_t o_ukey = take(sizeof(int32_t) * n_units);
    const size_t o_urank = take(sizeof(int32_t) * n_units);
    const size_t o_hist = take(sizeof(int32_t) * n_tiles * kKeys);
    const size_t o_order = take(sizeof(int32_t) * n_units);
    const size_t o_ktot = take(sizeof(int32_t) * kKeys);
    const size_t o_kbase = take(sizeof(int32_t) * kKeys);
    const size_t o_cpre = take(sizeof(int64_t) * (n_units + 1));
    const size_t o_ipre = take(sizeof(int64_t) * (n_units + 1));
    const size_t o_cval = take(sizeof(int64_t) * n_units);
    const size_t o_ival = take(sizeof(int64_t) * n_units);
    const size_t o_stmp = take(sizeof(int64_t) * scan_tmp_elems(n_units));
    const size_t o_chunks = take(sizeof(Chunk) * (n_units + 1));
    const size_t o_nch = take(sizeof(int32_t));
    const size_t o_perm = take(sizeof(int32_t) * N);
    char* mem = nullptr;
    SI_HIP(pool_alloc((void**)&mem, o, s));
    auto I = [&](size_t off) { return reinterpret_cast<int32_t*>(mem + off); };
    int32_t* perm0 = nullptr;
    hipError_t e = hipSuccess;
    if (sched->order != SI_ORDER_GIVEN && scene->n_cells > 1) {
        perm0 = I(o_perm0);
        e = launch_cell_order(oriented, N, *scene, I(o_key), I(o_rank), I(o_counts), I(o_starts),
                              I(o_tmp), perm0, s);
    }
    float* feats = reinterpret_cast<float*>(mem + o_feats);
    float* pred = reinterpret_cast<float*>(mem + o_pred);
    if (e == hipSuccess) {
        // features and predictions in loop order (perm0 applied here)
        SpinParams p;
        double R;
        if (make_params(params, &p, &R) != SI_OK) e = hipErrorInvalidValue;
        const SceneView v = view_of(*scene);
        int32_t* S = table ? reinterpret_cast<int32_t*>(mem + o_sat) : nullptr;
        if (e == hipSuccess && S) e = launch_sat(v, S, s);
        const float f11 = (float)(R / (kSub * scene->h));
        if (e == hipSuccess && S)
            hipLaunchKernelGGL(k_features_loop<true>, dim3(nblocks(N)), dim3(256), 0, s, v, S,
                               oriented, perm0, N, f11, feats);
        else if (e == hipSuccess)
            hipLaunchKernelGGL(k_features_loop<false>, dim3(nblocks(N)), dim3(256), 0, s, v, S,
                               oriented, perm0, N, f11, feats);
    }
    if (e == hipSuccess) {
        e = launch_mlp_predict_mfma(model->params, feats, N, pred, 0, s);
        hipLaunchKernelGGL(k_unit_cost, dim3(nblocks(n_units)), dim3(256), 0, s, pred, nullptr, N,
                           n_units, reinterpret_cast<uint32_t*>(mem + o_qcost), I(o_ukey));
        hipLaunchKernelGGL(k_unit_hist, dim3((unsigned)n_tiles), dim3(kTile), 0, s, I(o_ukey),
                           n_units, I(o_hist), I(o_urank));
        hipLaunchKernelGGL(k_unit_tile_scan, dim3(kKeys), dim3(256), 0, s, I(o_hist), (int)n_tiles,
                           I(o_ktot));
        hipLaunchKernelGGL(k_unit_key_base, dim3(1), dim3(kKeys), 0, s, I(o_ktot), I(o_kbase));
        hipLaunchKernelGGL(k_unit_scatter, dim3(nblocks(n_units)), dim3(256), 0, s, I(o_ukey),
                           I(o_urank), I(o_hist), I(o_kbase), n_units, I(o_order));
        auto L = [&](size_t off) { return reinterpret_cast<int64_t*>(mem + off); };
        hipLaunchKernelGGL(k_unit_gather, dim3(nblocks(n_units)), dim3(256), 0, s, I(o_order),
                           reinterpret_cast<uint32_t*>(mem + o_qcost), n_units, N, L(o_cval),
                           L(o_ival));
        if (e == hipSuccess) e = launch_scan64(L(o_cval), L(o_cpre), n_units, L(o_stmp), s);
        if (e == hipSuccess) e = launch_scan64(L(o_ival), L(o_ipre), n_units, L(o_stmp), s);
        hipLaunchKernelGGL(k_learned_chunks, dim3(1), dim3(1024), 0, s, L(o_cpre), L(o_ipre),
                           n_units, n_wg, sched->fac_divisor,
                           reinterpret_cast<Chunk*>(mem + o_chunks), I(o_nch));
        hipLaunchKernelGGL(k_learned_perm, dim3(nblocks(n_units)), dim3(256), 0, s, I(o_order),
                           reinterpret_cast<int64_t*>(mem + o_ipre), perm0, N, n_units, I(o_perm));
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e != hipSuccess) {
        (void)hipFreeAsync(mem, s);
        return hip_fail(e, "learned schedule");
    }
    plan->mem = mem;
    plan->chunks = reinterpret_cast<Chunk*>(mem + o_chunks);
    plan->max_chunks = (int32_t)(n_units + 1);
    plan->n_chunks_dev = I(o_nch);
    plan->perm = I(o_perm);
    return SI_OK;
}

int64_t learned_units(const int64_t* item_N, int n_items, int64_t* unit_off) {
    int64_t u = 0;
    for (int i = 0; i < n_items; ++i) {
        if (unit_off) unit_off[i] = u;
        u += (item_N[i] + kUnit - 1) / kUnit;
    }
    if (unit_off) unit_off[n_items] = u;
    return u;
}

bool use_feature_table(const int32_t* dims, int64_t N) {
    // measured on clustered2m: about 6 ns per table entry to build, then 33 ns
    // per image, against 123 ns per image summing grid rows
    if (const char* f = getenv("SI_FEATURES_TABLE")) {
        if (!strcmp(f, "always")) return true;
        if (!strcmp(f, "never")) return false;
    }
    return sat_entries(dims) <= 15 * N;
}

int64_t sat_offsets(const Item* items, int n_items, int64_t* off) {
    int64_t* e = off;
    int64_t* y = off + (n_items + 1);
    int64_t* z = off + 2 * (n_items + 1);
    e[0] = y[0] = z[0] = 0;
    for (int i = 0; i < n_items; ++i) {
        const int32_t* d = items[i].scene.dims;
        const bool t = use_feature_table(d, items[i].N);
        e[i + 1] = e[i] + (t ? sat_entries(d) : 0);
        y[i + 1] = y[i] + (t ? (int64_t)(d[0] + 1) * (d[2] + 1) : 0);
        z[i + 1] = z[i] + (t ? (int64_t)(d[0] + 1) * (d[1] + 1) : 0);
    }
    return e[n_items];
}

size_t learned_multi_layout(int n_items, int64_t total_N, int64_t n_units, int P,
                            const int64_t sat_pass[3], LearnedMulti& b, char* base) {
    const int64_t sat_total = sat_pass[0];
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + o : nullptr;
        o += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
        return p;
    };
    const int64_t n_tiles = (n_units + kTile - 1) / kTile;
    const size_t ik = (size_t)n_items * kKeys;
    b.unit_off = (int64_t*)take(sizeof(int64_t) * (n_items + 1));
    b.f11 = (float*)take(sizeof(float) * n_items);
    b.feats = (float*)take(sizeof(float) * kNF * total_N);
    b.pred = (float*)take(sizeof(float) * total_N);
    b.qcost = (uint32_t*)take(sizeof(uint32_t) * n_units);
    b.ukey = (int32_t*)take(sizeof(int32_t) * n_units);
    b.ulen = (int32_t*)take(sizeof(int32_t) * n_units);
    b.uitem = (int32_t*)take(sizeof(int32_t) * n_units);
    b.urank = (int32_t*)take(sizeof(int32_t) * n_units);
    b.hist = (int32_t*)take(sizeof(int32_t) * n_tiles * kKeys);
    b.ktot = (int32_t*)take(sizeof(int32_t) * kKeys);
    b.kbase = (int32_t*)take(sizeof(int32_t) * kKeys);
    b.order = (int32_t*)take(sizeof(int32_t) * n_units);
    b.cval = (int64_t*)take(sizeof(int64_t) * n_units);
    b.ival = (int64_t*)take(sizeof(int64_t) * n_units);
    b.cpre = (int64_t*)take(sizeof(int64_t) * (n_units + 1));
    b.ipre = (int64_t*)take(sizeof(int64_t) * (n_units + 1));
    b.ltmp = (int64_t*)take(sizeof(int64_t) * scan_tmp_elems(n_units + 1));
    b.ends = (int64_t*)take(sizeof(int64_t) * (P + 1));
    b.cut = (int32_t*)take(sizeof(int32_t) * n_units);
    b.hcount = (int32_t*)take(sizeof(int32_t) * ik);
    b.hlen = (int32_t*)take(sizeof(int32_t) * ik);
    b.base_len = (int32_t*)take(sizeof(int32_t) * ik);
    b.seg_first = (int32_t*)take(sizeof(int32_t) * ik);
    b.offs = (int32_t*)take(sizeof(int32_t) * n_units);
    b.flag = (int32_t*)take(sizeof(int32_t) * n_units);
    b.fpre = (int32_t*)take(sizeof(int32_t) * (n_units + 1));
    b.itmp = (int32_t*)take(sizeof(int32_t) * scan_tmp_elems(n_units + 1));
    b.perm = (int32_t*)take(sizeof(int32_t) * total_N);
    b.chunks = (Chunk*)take(sizeof(Chunk) * n_units);
    b.n_chunks = (int32_t*)take(sizeof(int32_t));
    b.sat_off = (int64_t*)take(sizeof(int64_t) * 3 * (n_items + 1));
    b.sat = (int32_t*)take(sizeof(int32_t) * sat_total);
    for (int k = 0; k < 3; ++k) b.sat_pass[k] = sat_pass[k];
    return o;
}

hipError_t learned_multi_enqueue(const si_cost_model* model, const LearnedMulti& b,
                                 const Item* items, const int64_t* item_off, int n_items,
                                 const int32_t* perm_cell, int64_t total_N, int64_t n_units, int P,
                                 float divisor, hipStream_t s) {
    const int64_t n_tiles = (n_units + kTile - 1) / kTile;
    const int64_t ik = (int64_t)n_items * kKeys;
    hipError_t e = launch_fill(b.hcount, ik, 0, s);
    if (e == hipSuccess) e = launch_fill(b.hlen, ik, 0, s);
    if (e == hipSuccess) e = launch_fill(b.cut, n_units, 0, s);
    if (e != hipSuccess) return e;
    e = launch_features_multi(items, item_off, n_items, perm_cell, b.f11, b.sat_off, b.sat,
                              b.sat_pass, total_N, b.feats, s);
    if (e != hipSuccess) return e;
    e = launch_mlp_predict_mfma(model->params, b.feats, total_N, b.pred, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_unit_cost_multi, dim3(nblocks(n_units)), dim3(256), 0, s, b.pred,
                       b.unit_off, item_off, n_items, n_units, b.qcost, b.ukey, b.ulen, b.uitem,
                       b.hcount, b.hlen);
    // one LPT order of all units (stable by key)
    hipLaunchKernelGGL(k_unit_hist, dim3((unsigned)n_tiles), dim3(kTile), 0, s, b.ukey, n_units,
                       b.hist, b.urank);
    hipLaunchKernelGGL(k_unit_tile_scan, dim3(kKeys), dim3(256), 0, s, b.hist, (int)n_tiles,
                       b.ktot);
    hipLaunchKernelGGL(k_unit_key_base, dim3(1), dim3(kKeys), 0, s, b.ktot, b.kbase);
    hipLaunchKernelGGL(k_unit_scatter, dim3(nblocks(n_units)), dim3(256), 0, s, b.ukey, b.urank,
                       b.hist, b.kbase, n_units, b.order);
    hipLaunchKernelGGL(k_unit_gather_multi, dim3(nblocks(n_units)), dim3(256), 0, s, b.order,
                       b.qcost, b.ulen, n_units, b.cval, b.ival);
    e = launch_scan64(b.cval, b.cpre, n_units, b.ltmp, s);
    if (e == hipSuccess) e = launch_scan64(b.ival, b.ipre, n_units, b.ltmp, s);
    if (e != hipSuccess) return e;
    // global chunks by factoring on cost, then each item's new order
    hipLaunchKernelGGL(k_learned_cuts, dim3(1), dim3(1024), 0, s, b.cpre, n_units, P, divisor,
                       b.ends, b.cut);
    hipLaunchKernelGGL(k_item_key_base, dim3((unsigned)n_items), dim3(kKeys), 0, s, b.hlen,
                       b.base_len);
    hipLaunchKernelGGL(k_seg_first, dim3(kKeys), dim3(256), 0, s, b.hcount, b.kbase, n_items,
                       b.seg_first);
    hipLaunchKernelGGL(k_learned_perm_multi, dim3(nblocks(n_units)), dim3(256), 0, s, b.order,
                       b.ukey, b.ulen, b.uitem, b.unit_off, item_off, n_items, b.ipre, b.base_len,
                       b.seg_first, b.cut, perm_cell, n_units, b.offs, b.flag, b.perm);
    e = launch_scan(b.flag, b.fpre, n_units, b.itmp, scan_tmp_elems(n_units), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_emit_runs, dim3(nblocks(n_units)), dim3(256), 0, s, b.order, b.uitem,
                       b.ulen, b.offs, b.flag, b.fpre, n_units, b.chunks, b.n_chunks);
    return hipGetLastError();
}

uint64_t model_serial(const si_cost_model* m) { return m ? m->serial : 0; }

}  // namespace si

using namespace si;

extern "C" {

si_status si_features(const si_scene* scene, const int32_t* oriented_idx, int64_t N,
                      const si_params* params, float* feats_out, void* hip_stream) {
    if (!scene || (N > 0 && (!oriented_idx || !feats_out))) return fail(SI_E_INVALID, "NULL argument");
    if (N < 0 || N >= INT32_MAX) return fail(SI_E_INVALID, "N out of range");
    if (N == 0) return SI_OK;
    return features_launch(*scene, oriented_idx, N, params, feats_out, (hipStream_t)hip_stream);
}

si_status si_cost_model_create(uint64_t seed, si_cost_model** out) {
    if (!out) return fail(SI_E_INVALID, "out is NULL");
    *out = nullptr;
    si_cost_model* m = new (std::nothrow) si_cost_model();
    if (!m) return fail(SI_E_OOM, "host allocation failed");
    m->seed = seed;
    SI_HIP(hipGetDevice(&m->device));
    // He-uniform weights (bound sqrt(6 / fan_in)), zero biases
    std::vector<float> h(kNP, 0.0f);
    uint64_t st = seed ^ 0x5eed5eed5eed5eedull;
    auto fill = [&](int off, int n, int fan_in) {
        const double bound = sqrt(6.0 / fan_in);
        for (int i = 0; i < n; ++i) h[off + i] = (float)((2.0 * uniform01(st) - 1.0) * bound);
    };
    fill(oW1, kH * kNF, kNF);
    fill(oW2, kH * kH, kH);
    fill(oW3, kH, kH);
    hipError_t e = hipMalloc(&m->params, sizeof(float) * kNP);
    if (e == hipSuccess) e = hipMalloc(&m->m, sizeof(float) * kNP);
    if (e == hipSuccess) e = hipMalloc(&m->v, sizeof(float) * kNP);
    if (e == hipSuccess) e = hipMemcpy(m->params, h.data(), sizeof(float) * kNP, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->m, 0, sizeof(float) * kNP);
    if (e == hipSuccess) e = hipMemset(m->v, 0, sizeof(float) * kNP);
    if (e != hipSuccess) {
        si_free_cost_model(m);
        return hip_fail(e, "cost model allocation");
    }
    *out = m;
    return SI_OK;
}

void si_free_cost_model(si_cost_model* m) {
    if (!m) return;
    si::drop_graphs_of(m->serial);
    (void)hipFree(m->params);
    (void)hipFree(m->m);
    (void)hipFree(m->v);
    delete m;
}

si_status si_cost_model_gradient(const si_cost_model* m, const float* feats, const uint32_t* counts,
                                 int64_t n, float* grad_host, float* loss_host, void* hip_stream) {
    if (!m || !feats || !counts || n <= 0) return fail(SI_E_INVALID, "bad arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    const int nblk = (int)((n + kGradSamples - 1) / kGradSamples);
    float* mem = nullptr;
    SI_HIP(pool_alloc((void**)&mem, sizeof(float) * ((size_t)nblk * (kNP + 1) + kNP + 1), s));
    float* part = mem;
    float* grad = mem + (size_t)nblk * (kNP + 1);
    float* loss = grad + kNP;
    hipError_t e = launch_fill(reinterpret_cast<int32_t*>(loss), 1, 0, s);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), 0, s, m->params, feats, counts,
                       (const int32_t*)nullptr, (int64_t)0, n, (float)(1.0 / (double)n), part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(nblocks(kNP + 1)), dim3(256), 0, s, part, nblk, grad, loss);
    if (e == hipSuccess) e = hipGetLastError();
    std::vector<float> h(kNP + 1);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), grad, sizeof(float) * (kNP + 1), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(mem, s);
    if (e != hipSuccess) return hip_fail(e, "cost model gradient");
    if (grad_host) memcpy(grad_host, h.data(), sizeof(float) * kNP);
    if (loss_host) *loss_host = h[kNP] / (float)n;
    return SI_OK;
}

si_status si_cost_model_train(si_cost_model* m, const float* feats, const uint32_t* counts, int64_t n,
                              int32_t epochs, float lr, int32_t batch, float* loss_curve_host,
                              void* hip_stream) {
    if (!m || !feats || !counts || n <= 0) return fail(SI_E_INVALID, "bad arguments");
    if (epochs < 0 || batch < 1 || batch > 65536 || !(lr > 0.0f) || !isfinite(lr))
        return fail(SI_E_INVALID, "epochs >= 0, 1 <= batch <= 65536, lr > 0 required");
    if (n >= INT32_MAX) return fail(SI_E_INVALID, "n out of range");
    hipStream_t s = (hipStream_t)hip_stream;
    const int nblk_max = (batch + kGradSamples - 1) / kGradSamples;
    size_t words = (size_t)nblk_max * (kNP + 1) + kNP + (size_t)std::max(epochs, 1) + (size_t)n;
    float* mem = nullptr;
    SI_HIP(pool_alloc((void**)&mem, sizeof(float) * words, s));
    float* part = mem;
    float* grad = part + (size_t)nblk_max * (kNP + 1);
    float* losses = grad + kNP;
    int32_t* perm = reinterpret_cast<int32_t*>(losses + std::max(epochs, 1));
    int32_t* hperm = nullptr;
    hipError_t e = hipHostMalloc((void**)&hperm, sizeof(int32_t) * n, hipHostMallocDefault);
    if (e == hipSuccess) e = launch_fill(reinterpret_cast<int32_t*>(losses), std::max(epochs, 1), 0, s);
    uint64_t rng = m->seed * 0x2545f4914f6cdd1dull + 12345;
    for (int32_t ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        // the previous epoch's copy of hperm must be complete before refilling it
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) break;
        for (int64_t i = 0; i < n; ++i) hperm[i] = (int32_t)i;
        for (int64_t i = n - 1; i > 0; --i) {
            const int64_t j = (int64_t)(splitmix(rng) % (uint64_t)(i + 1));
            std::swap(hperm[i], hperm[j]);
        }
        e = hipMemcpyAsync(perm, hperm, sizeof(int32_t) * n, hipMemcpyHostToDevice, s);
        for (int64_t b0 = 0; b0 < n && e == hipSuccess; b0 += batch) {
            const int64_t cnt = std::min<int64_t>(batch, n - b0);
            const int nblk = (int)((cnt + kGradSamples - 1) / kGradSamples);
            hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), 0, s, m->params, feats, counts,
                               perm, b0, cnt, (float)(1.0 / (double)cnt), part);
            hipLaunchKernelGGL(k_mlp_reduce, dim3(nblocks(kNP + 1)), dim3(256), 0, s, part, nblk,
                               grad, losses + ep);
            ++m->step;
            const float bc1 = (float)(1.0 - pow(0.9, (double)m->step));
            const float bc2 = (float)(1.0 - pow(0.999, (double)m->step));
            hipLaunchKernelGGL(k_adam, dim3(nblocks(kNP)), dim3(256), 0, s, m->params, grad, m->m,
                               m->v, lr, bc1, bc2);
            e = hipGetLastError();
        }
    }
    std::vector<float> hl(std::max(epochs, 1));
    if (e == hipSuccess && loss_curve_host && epochs > 0)
        e = hipMemcpyAsync(hl.data(), losses, sizeof(float) * epochs, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(mem, s);
    if (hperm) (void)hipHostFree(hperm);
    if (e != hipSuccess) return hip_fail(e, "cost model training");
    if (loss_curve_host)
        for (int32_t ep = 0; ep < epochs; ++ep) loss_curve_host[ep] = hl[ep] / (float)n;
    return SI_OK;
}

si_status si_cost_model_predict(const si_cost_model* m, const float* feats, int64_t n,
                                float* pred_counts, void* hip_stream) {
    if (!m || (n > 0 && (!feats || !pred_counts))) return fail(SI_E_INVALID, "bad arguments");
    if (n <= 0) return SI_OK;
    hipLaunchKernelGGL(k_mlp_predict, dim3(nblocks(n)), dim3(256), 0, (hipStream_t)hip_stream,
                       m->params, feats, n, pred_counts, 0);
    SI_HIP(hipGetLastError());
    return SI_OK;
}

si_status si_cost_model_predict_planner(const si_cost_model* m, const float* feats, int64_t n,
                                        float* pred_counts, void* hip_stream) {
    if (!m || (n > 0 && (!feats || !pred_counts))) return fail(SI_E_INVALID, "bad arguments");
    if (n <= 0) return SI_OK;
    if (reinterpret_cast<uintptr_t>(feats) & 15)
        return fail(SI_E_INVALID, "feats must be 16-byte aligned");
    SI_HIP(launch_mlp_predict_mfma(m->params, feats, n, pred_counts, 0, (hipStream_t)hip_stream));
    return SI_OK;
}

si_status si_cost_model_get_params(const si_cost_model* m, float* host_params, int64_t n) {
    if (!m || !host_params || n != kNP) return fail(SI_E_INVALID, "need a buffer of 5057 floats");
    SI_HIP(hipMemcpy(host_params, m->params, sizeof(float) * kNP, hipMemcpyDeviceToHost));
    return SI_OK;
}

si_status si_cost_model_set_params(si_cost_model* m, const float* host_params, int64_t n) {
    if (!m || !host_params || n != kNP) return fail(SI_E_INVALID, "need a buffer of 5057 floats");
    SI_HIP(hipMemcpy(m->params, host_params, sizeof(float) * kNP, hipMemcpyHostToDevice));
    SI_HIP(hipMemset(m->m, 0, sizeof(float) * kNP));
    SI_HIP(hipMemset(m->v, 0, sizeof(float) * kNP));
    m->step = 0;
    return SI_OK;
}

// File: "SICM" magic, uint32 version 1, uint32 parameter count, uint64 seed,
// then the parameters as little-endian float32.
si_status si_cost_model_save(const si_cost_model* m, const char* path) {
    if (!m || !path) return fail(SI_E_INVALID, "NULL argument");
    std::vector<float> h(kNP);
    si_status rc = si_cost_model_get_params(m, h.data(), kNP);
    if (rc != SI_OK) return rc;
    FILE* f = fopen(path, "wb");
    if (!f) return fail(SI_E_INVALID, std::string("cannot open ") + path);
    const uint32_t ver = 1, np = kNP;
    bool ok = fwrite("SICM", 1, 4, f) == 4 && fwrite(&ver, 4, 1, f) == 1 && fwrite(&np, 4, 1, f) == 1 &&
              fwrite(&m->seed, 8, 1, f) == 1 && fwrite(h.data(), 4, kNP, f) == (size_t)kNP;
    ok = (fclose(f) == 0) && ok;
    return ok ? SI_OK : fail(SI_E_INVALID, "write failed");
}

si_status si_cost_model_load(const char* path, si_cost_model** out) {
    if (!path || !out) return fail(SI_E_INVALID, "NULL argument");
    *out = nullptr;
    FILE* f = fopen(path, "rb");
    if (!f) return fail(SI_E_INVALID, std::string("cannot open ") + path);
    char magic[4];
    uint32_t ver = 0, np = 0;
    uint64_t seed = 0;
    std::vector<float> h(kNP);
    bool ok = fread(magic, 1, 4, f) == 4 && memcmp(magic, "SICM", 4) == 0 && fread(&ver, 4, 1, f) == 1 &&
              ver == 1 && fread(&np, 4, 1, f) == 1 && np == (uint32_t)kNP && fread(&seed, 8, 1, f) == 1 &&
              fread(h.data(), 4, kNP, f) == (size_t)kNP;
    fclose(f);
    if (!ok) return fail(SI_E_INVALID, "not a cost-model file");
    for (float x : h)
        if (!isfinite(x)) return fail(SI_E_INVALID, "cost-model file holds non-finite parameters");
    si_status rc = si_cost_model_create(seed, out);
    if (rc != SI_OK) return rc;
    rc = si_cost_model_set_params(*out, h.data(), kNP);
    if (rc != SI_OK) {
        si_free_cost_model(*out);
        *out = nullptr;
    }
    return rc;
}

si_status si_learned_table(const float* unit_cost, int64_t n, int32_t P, float fac_divisor,
                           int32_t* perm_out, int64_t* starts_out, int64_t cap, int64_t* n_chunks) {
    // Host reference of the ordering and cutting the device computes (for
    // inspection and tests): units in descending cost key (stable), then
    // factoring on cost.  unit_cost are already-rounded positive costs.
    if (!unit_cost || n < 0 || P < 1 || !perm_out || !starts_out || !n_chunks)
        return fail(SI_E_INVALID, "bad arguments");
    std::vector<uint32_t> q(n);
    std::vector<int32_t> key(n);
    for (int64_t u = 0; u < n; ++u) {
        const float c = unit_cost[u];
        q[u] = (uint32_t)std::max(rintf(c == c ? std::min(c, 4.0e9f) : 1.0f), 1.0f);
        const int k = (int)floorf(log2f((float)q[u]) * 32.0f);
        key[u] = kKeys - 1 - std::min(std::max(k, 0), kKeys - 1);
    }
    std::vector<int32_t> order(n);
    for (int64_t u = 0; u < n; ++u) order[u] = (int32_t)u;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    std::vector<int64_t> cpre(n + 1, 0);
    for (int64_t k = 0; k < n; ++k) cpre[k + 1] = cpre[k] + q[order[k]];
    const double x = fac_divisor > 0.0f ? (double)fac_divisor : 2.0;
    std::vector<int64_t> starts;
    starts.push_back(0);
    int64_t st = 0;
    while (st < n) {
        const int64_t R = cpre[n] - cpre[st];
        const int64_t cb = std::max<int64_t>(1, (int64_t)ceil((double)R / (x * (double)P)));
        int64_t prev = st;
        for (int j = 1; j <= P; ++j) {
            const int64_t target = cpre[st] + (int64_t)j * cb;
            const int64_t e = std::lower_bound(cpre.begin() + st + 1, cpre.end() - 1 + 1, target) -
                              cpre.begin();
            const int64_t end = std::min<int64_t>(e, n);
            if (end > prev) {
                starts.push_back(end);
                prev = end;
            }
        }
        st = prev;
    }
    *n_chunks = (int64_t)starts.size() - 1;
    for (int64_t u = 0; u < n; ++u) perm_out[u] = order[u];
    if (cap < (int64_t)starts.size()) return fail(SI_E_INVALID, "starts_out capacity too small");
    for (size_t i = 0; i < starts.size(); ++i) starts_out[i] = starts[i];
    return SI_OK;
}

}  // extern "C"
