// Helpers shared by the C ABI translation units (api.cpp and the batched
// and serving front ends): error state, argument conversion, sizing.
#pragma once

#include <cstdarg>
#include <cstddef>
#include <cstdint>

#include "../../include/gs.h"
#include "gs_device.h"
#include "kernels.h"

namespace gs {

constexpr int64_t kMaxPairs = (1ll << 30) - 1;

// Record `fmt` as this thread's last error and return `code`.
gs_status fail(gs_status code, const char* fmt, ...);
const char* g_err_cstr();
// GS_ERR_HIP with the runtime's message if the last launch failed.
gs_status check_hip(const char* what);

gs_status to_cam(const gs_camera* c, Cam* out);
gs_status to_gauss(const gs_gaussians* g, Gauss* out);
gs_status tiles_of(const gs_opts* o, int* tw, int* th);
int tile_bits(int64_t n_tiles);
size_t align256(size_t x);
size_t bin_sort_ws_bytes(int64_t n, int64_t cap, int64_t n_tiles);
gs_status check_proj(const gs_proj* p, int64_t n);
gs_status check_bins(const gs_bins* b);

// One-entry view / job tables and blend arguments of the single-view calls.
ViewTab single_view(const Cam& C, int tw, int th);
JobTab single_job(const Gauss& G, const gs_grads* out);
RenderArgs single_render(const gs_proj* proj, const gs_bins* bins, const Cam& C, int tw, int th);

}  // namespace gs
