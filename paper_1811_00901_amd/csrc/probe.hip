// Peak probes: the throughput ceilings that the spin kernel's roofline is
// read against, measured on the device that runs it (a published peak is a
// bound; these are what the hardware delivers to such code).
//
//   VALU          FP32 fused multiply-adds, 16 independent chains per lane
//                 (one lane-operation each), no packed instructions
//   LDS atomics   ds_add_u32 on a 4,096-word array: 64 consecutive words per
//                 wave-instruction (conflict free), or 64 random words of a
//                 W^2 = 1,024 image (the binning pattern)
//   HBM           a float4 copy of 1 GiB into 1 GiB; bytes read + written
#include "si_internal.h"

namespace si {

namespace {

constexpr int kProbeBlock = 256;

__global__ void __launch_bounds__(kProbeBlock) k_probe_valu(float* __restrict__ out, int iters,
                                                            float a, float b) {
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = (float)threadIdx.x * 1e-3f + (float)k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = fmaf(v[k], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += v[k];
    if (s == 1234.5f) out[blockIdx.x] = s;  // keeps the chains alive
}

// 16 atomics per round at base + 67 k (random) or base + 64 k (sequential).
__global__ void __launch_bounds__(kProbeBlock) k_probe_lds(uint32_t* __restrict__ out, int rounds,
                                                           int random) {
    __shared__ uint32_t bins[4096 + 16 * 67];
    for (int i = threadIdx.x; i < 4096 + 16 * 67; i += kProbeBlock) bins[i] = 0u;
    __syncthreads();
    uint32_t x = threadIdx.x * 2654435761u + blockIdx.x * 40503u + 1u;
    for (int r = 0; r < rounds; ++r) {
        uint32_t base;
        if (random) {
            x = x * 1664525u + 1013904223u;
            base = x >> 22;  // 0 .. 1023
        } else {
            base = (threadIdx.x & 63) + 64u * (threadIdx.x >> 6);
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) atomicAdd(&bins[base + (random ? 67u : 256u) * k], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0 && bins[1] == 0xFFFFFFFFu) out[blockIdx.x] = bins[0];
}

__global__ void __launch_bounds__(kProbeBlock) k_probe_copy(const float4* __restrict__ src,
                                                            float4* __restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kProbeBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kProbeBlock)
        dst[i] = src[i];
}

}  // namespace

}  // namespace si

using namespace si;

extern "C" si_status si_peak_probe(int32_t kind, double* value, void* hip_stream) {
    if (!value) return fail(SI_E_INVALID, "value is NULL");
    if (kind < SI_PROBE_VALU || kind > SI_PROBE_HBM_COPY) return fail(SI_E_INVALID, "bad probe kind");
    hipStream_t s = (hipStream_t)hip_stream;
    DeviceState* st;
    si_status rc = device_state(&st);
    if (rc != SI_OK) return rc;
    const int blocks = st->n_cu * 8;
    const size_t copy_elems = (size_t)1 << 26;  // 64 Mi float4 = 1 GiB
    char* mem = nullptr;
    const size_t bytes = kind == SI_PROBE_HBM_COPY ? 2 * copy_elems * sizeof(float4)
                                                   : sizeof(float) * (size_t)blocks;
    SI_HIP(hipMallocAsync((void**)&mem, bytes, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int valu_iters = 16384, lds_rounds = 4096;
    auto launch = [&]() {
        if (kind == SI_PROBE_VALU)
            hipLaunchKernelGGL(k_probe_valu, dim3(blocks), dim3(kProbeBlock), 0, s,
                               reinterpret_cast<float*>(mem), valu_iters, 0.999f, 1e-3f);
        else if (kind == SI_PROBE_HBM_COPY)
            hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(kProbeBlock), 0, s,
                               reinterpret_cast<const float4*>(mem),
                               reinterpret_cast<float4*>(mem) + copy_elems, (int64_t)copy_elems);
        else
            hipLaunchKernelGGL(k_probe_lds, dim3(blocks), dim3(kProbeBlock), 0, s,
                               reinterpret_cast<uint32_t*>(mem), lds_rounds,
                               kind == SI_PROBE_LDS_ATOMIC_RANDOM ? 1 : 0);
        return hipGetLastError();
    };
    float ms = 0.0f;
    if (e == hipSuccess && kind == SI_PROBE_HBM_COPY)
        e = hipMemsetAsync(mem, 0, copy_elems * sizeof(float4), s);
    if (e == hipSuccess) e = launch();  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFreeAsync(mem, s);
    if (e != hipSuccess) return hip_fail(e, "peak probe");
    const double threads = (double)blocks * kProbeBlock;
    double work = 0.0;
    if (kind == SI_PROBE_VALU) work = threads * valu_iters * 16.0;
    else if (kind == SI_PROBE_HBM_COPY) work = 2.0 * (double)copy_elems * sizeof(float4);
    else work = threads * lds_rounds * 16.0;
    *value = work / ((double)ms * 1e-3);
    return SI_OK;
}
