// sfft_host.h -- host-side pieces shared by the C-ABI driver and the serving
// loop: the workspace layout of a batch, its binding to device memory, and
// the launch sequence of one pipeline (not part of the public ABI).
#pragma once

#include <vector>

#include "sfft_internal.h"

namespace sfft {

struct LevelLaunch {
  bool fft, direct, children, jump, col;
  int grid_fft, grid_direct, grid_children, grid_jump, grid_resolve, grid_col, grid_col_resolve, grid_col_deep;
};

// Workspace of one batch, decided on the host from its plans alone: every
// signal's descriptor with its offsets into the arenas, the work lists, the
// size of every arena and its byte offset in one device slab, and the static
// launch shape of every tree level.  No device call.
struct Layout {
  std::vector<SigDesc> desc;
  std::vector<int32_t> lists;
  int ntree = 0, nffast = 0;
  size_t l0_at = 0, l0c_at = 0;
  int32_t l0_items = 0, l0c_items = 0;
  int nmax = 1, max_B0 = 1, max_stage = 1, max_found_cap = 64;
  int32_t jrows = kJumpItemRows, any_fp32 = 0, col_lp_mask = 0, col_f16_mask = 0, col16_mask = 0,
          any_wide_jump = 0,
          any_noisy0 = 0, any_noisy = 0, any_noise_est = 0, l0_spread_lg = 0, gather_u = 4, l0_lds = 16,
          deep_lds = 0;
  bool any_jump = false;
  std::vector<LevelLaunch> levels;
  // arena sizes in elements
  int64_t n_y0 = 0, n_fst = 0, n_found = 0, n_multi = 0, n_mvec = 0, n_jacc = 0, n_jcol = 0;
  // byte offsets of the parts of the slab, and its size
  size_t o_desc = 0, o_io = 0, o_st = 0, o_lists = 0, o_pre = 0, o_out = 0, o_y0 = 0, o_fst = 0,
         o_ff = 0, o_fa = 0, o_mc = 0, o_my = 0, o_mz = 0, o_jacc = 0, o_jcol = 0, o_deep = 0, bytes = 0;
};

// Timing events of a profiled pipeline run: one after every launch, with the
// kernel id of each interval.
struct Prof {
  std::vector<hipEvent_t> ev;
  std::vector<int32_t> id;
};

// Workspace of the batch of plans ps (host only); ncu sizes the persistent grids.
int32_t make_layout(const std::vector<const sfft_plan_s *> &ps, bool no_jump, int ncu, Layout &Y);
// Launch context of layout Y placed at `base` (a device slab of Y.bytes whose
// descriptor and list parts hold Y.desc and Y.lists).
void bind_layout(const Layout &Y, char *base, const float2 *tw, LaunchCtx &c);
// The whole pipeline of a layout bound in c, on stream s (timing events with prof).
hipError_t launch_pipeline(const Layout &lay, const LaunchCtx &c, hipStream_t s, Prof *prof);
// Per-device twiddle table e^{-2 pi i k / kFftMax} (allocated once per device).
hipError_t device_twiddles(int dev, const float2 **out);
int device_cus(int device);
bool is_device_ptr(const void *p);
// sets the calling thread's last error code and returns it
int32_t set_last_error(int32_t code);

}  // namespace sfft
