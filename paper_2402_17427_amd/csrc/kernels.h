// Host-side launchers of the rasterizer kernels.  Each enqueues on `st`
// and returns at once; shapes are validated by the C ABI layer (api.cpp)
// before any of these is called.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gs_device.h"

namespace gs {

// ---- projection (project.hip)
void launch_project(const Gauss& g, const Cam& cam, int tw, int th, Rec* rec, float* depth, ushort4* rect,
                    uint32_t* tiles_touched, hipStream_t st);
void launch_project_bwd(const Gauss& g, const Cam& cam, const uint32_t* tiles_touched, const float* g2d,
                        const int32_t* status, int64_t gld, float* gmean, float* gscale, float* gquat, float* gopac,
                        float* gsh, hipStream_t st);

// ---- binning (binning.hip)
// Workspace for the tiles_touched scan over n Gaussians.
size_t scan_workspace_bytes(int64_t n);
// Exclusive scan of tiles_touched, then one (tile << 32 | depth bits, index)
// pair per covered tile.  Writes *pair_count and sets *status to
// GS_ERR_CAPACITY (-4) when the pairs exceed `capacity` (pairs beyond it
// are dropped).
void launch_emit_pairs(int64_t n, const uint32_t* tiles_touched, const ushort4* rect, const float* depth,
                       int ntx, int64_t capacity, uint64_t* keys, uint32_t* vals, uint32_t* pair_count,
                       int32_t* status, void* scan_ws, hipStream_t st);
void launch_tile_ranges(const uint64_t* keys, const uint32_t* pair_count, int64_t capacity, int64_t n_tiles,
                        uint32_t* ranges, hipStream_t st);
void launch_fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t st);

// ---- radix sort (sort.hip)
size_t sort_workspace_bytes(int64_t capacity, int key_bits);
// Stable LSD sort of (key, val) on the low key_bits bits.  The sorted pairs
// end in (keys, vals); (alt_keys, alt_vals) are ping-pong buffers of the
// same capacity.  When `start_in_alt` is set the input is read from the
// alternate buffers instead (so that an odd pass count still ends in
// keys/vals).
int sort_passes(int key_bits);
void launch_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* alt_keys, uint32_t* alt_vals,
                       const uint32_t* count, int64_t capacity, int key_bits, bool start_in_alt, void* ws,
                       hipStream_t st);

// ---- blend (render_fwd.hip / render_bwd.hip)
bool render_tile_supported(int tw, int th);
// stats != NULL runs the counting variant instead (no image written);
// state != NULL also stores the per-entry blend state (P * tile pixels).
void launch_render_fwd(const Rec* rec, const uint32_t* vals, const uint32_t* ranges, const int32_t* status,
                       const Cam& cam, int tw, int th, float* image, float* final_T, uint32_t* n_contrib,
                       unsigned long long* stats, float2* state, hipStream_t st);
// state != NULL reads the stored blend state instead of recomputing it.
void launch_render_bwd(const Rec* rec, const uint32_t* vals, const uint32_t* ranges, const int32_t* status,
                       const Cam& cam, int tw, int th, const float* final_T, const uint32_t* n_contrib,
                       const float* dimg, int64_t n, float* g2d, const float2* state, hipStream_t st);

}  // namespace gs
