// Declarations of the batched scene build (si_build_scenes), shared by the
// host runtime and the scene kernels.  Nothing here is part of the C ABI.
#pragma once

#include "si_internal.h"

namespace si {

// The grid a scene's points are binned with.
struct GridDesc {
    double origin[3];
    double h;
    int32_t dims[3];
};

// One scene of a batched build: its inputs, its grid, where its keys start
// in the concatenated key space, and its (library-owned) arrays.
struct BuildItem {
    const float* xyz;
    const float* nrm;
    int64_t M;
    GridDesc g;
    int64_t key_base;
    float4* pos;
    float4* nr;
    int32_t* inv;
    int32_t* sub_start;
};

// The grid a scene's points were binned with.
inline GridDesc grid_of(const Scene& sc) {
    GridDesc g;
    for (int a = 0; a < 3; ++a) {
        g.origin[a] = (double)sc.origin[a];
        g.dims[a] = sc.dims[a];
    }
    g.h = sc.h;
    return g;
}

// Bounding boxes of many scenes in two launches: scene s owns the partial
// blocks blk_off[s] <= b < blk_off[s+1] (every scene at least one); part
// holds 6 floats per block, out6 6 per scene (as launch_bbox).
hipError_t launch_bbox_multi(const BuildItem* items, const int64_t* blk_off, int n,
                             int64_t total_blocks, float* part, float* out6, hipStream_t s);
// Bin, scan and scatter many scenes at once.  Point t of the concatenation
// belongs to scene s with pt_off[s] <= t < pt_off[s+1]; sub_start entry t
// (n_keys_s + 1 per scene) to s with sub_off[s] <= t < sub_off[s+1].
// Temporaries: key_of, rank (total_M); counts (total_keys); gscan
// (total_keys + 1); tmp (scan_tmp_elems(total_keys)).
hipError_t launch_build_multi(const BuildItem* items, const int64_t* pt_off,
                              const int64_t* sub_off, int n, int64_t total_M, int64_t total_keys,
                              int32_t* key_of, int32_t* rank, int32_t* counts, int32_t* gscan,
                              int32_t* tmp, hipStream_t s);

}  // namespace si
