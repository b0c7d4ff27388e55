// sfft_host.cpp -- plans, batch contexts and the C-ABI of the aliasing-filter
// sparse FFT library (host side; the kernels live in sfft_kernels.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "sfft_host.h"

using namespace sfft;

namespace {

thread_local int32_t g_last_error = SFFT_OK;

int32_t fail(int32_t code) {
  g_last_error = code;
  return code;
}

bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) l++;
  return l;
}
int64_t npow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// SplitMix64 of Steele, Lea & Flood (OOPSLA 2014): Weyl increment by the
// 64-bit golden ratio, then the two xor-shift-multiply mixing steps.
struct SplitMix64 {
  uint64_t x;
  uint64_t next() {
    x += 0x9E3779B97F4A7C15ULL;
    uint64_t v = x;
    v ^= v >> 30;
    v *= 0xBF58476D1CE4E5B9ULL;
    v ^= v >> 27;
    v *= 0x94D049BB133111EBULL;
    v ^= v >> 31;
    return v;
  }
};

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

struct BatchCtx;
struct HostCtx;

}  // namespace

struct sfft_plan_s {
  sfft_plan_info_t info;
  int64_t stage_off[SFFT_MAX_STAGES + 1];
  int64_t nb;            // FFAST buckets (sum of stage sizes)
  double noise_p_den;
  int64_t noise_at;
  std::unique_ptr<BatchCtx> single;
  std::unique_ptr<HostCtx> host;   // host-gather solves (sfft_exec_host)
  std::unique_ptr<Layout> na_lay;  // sfft_exec_noalloc: layout of this plan alone
  int na_dev = -1;
};

namespace {

constexpr int64_t kMaxN = int64_t(1) << 30;
constexpr int32_t kBatchPrepareOnly = 1 << 16;  // internal flag of sfft_exec_batch_ex

// ------------------------------------------------------------ device buffers
struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) {
    if (p) (void)hipFree(p);
    p = nullptr;
    return hipMalloc(&p, bytes ? bytes : 16);
  }
};

}  // namespace

void sfft::host_twiddles(float2 *out) {
  for (int k = 0; k < kFftMax; k++) {
    const double a = 2.0 * M_PI * (double)k / (double)kFftMax;
    out[k] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
}

namespace sfft {

// per-device twiddle table e^{-2 pi i k / kFftMax}
std::mutex g_tw_mu;
std::map<int, float2 *> g_tw;

hipError_t device_twiddles(int dev, const float2 **out) {
  std::lock_guard<std::mutex> lk(g_tw_mu);
  auto it = g_tw.find(dev);
  if (it != g_tw.end()) {
    *out = it->second;
    return hipSuccess;
  }
  std::vector<float2> h(kFftMax);
  host_twiddles(h.data());
  float2 *d = nullptr;
  hipError_t e = hipMalloc(&d, sizeof(float2) * kFftMax);
  if (e != hipSuccess) return e;
  e = hipMemcpy(d, h.data(), sizeof(float2) * kFftMax, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  g_tw[dev] = d;
  *out = d;
  return hipSuccess;
}

// first tree level whose parents' stride N / (B0 2^{l-1}) is <= jump_L, or a
// level beyond max_levels when the subtree resolution is off
int jump_level(const SigDesc &d) {
  if (d.jump_L <= 0) return d.max_levels + 1;
  for (int l = 1; l <= d.max_levels; l++)
    if ((d.N >> (d.log2B0 + l - 1)) <= d.jump_L) return l;
  return d.max_levels + 1;
}

constexpr size_t kSlabAlign = 256;
size_t align_up(size_t v) { return (v + kSlabAlign - 1) & ~(kSlabAlign - 1); }

int32_t make_layout(const std::vector<const sfft_plan_s *> &ps, bool no_jump, int ncu, Layout &Y) {
  const int nsig = (int)ps.size();
  Y = Layout{};
  Y.desc.resize(nsig);
  int64_t y0 = 0, fst = 0, fc = 0, mc = 0, jc = 0;
  int nmax = 1, maxB0 = 1, maxStage = 1, maxFcap = 64;
  std::vector<std::pair<int64_t, int>> tree, ffast;
  for (int s = 0; s < nsig; s++) {
    const sfft_plan_s *p = ps[s];
    const sfft_plan_info_t &in = p->info;
    SigDesc d{};
    d.N = in.N;
    d.K = in.K;
    d.B0 = in.B0;
    d.log2N = pow2(in.N) ? ilog2(in.N) : -1;
    d.log2B0 = in.kind == SFFT_KIND_TREE ? ilog2(in.B0) : 0;
    d.kind = in.kind;
    d.mode = in.mode;
    d.R = in.R;
    d.D = in.D;
    d.n = in.kind == SFFT_KIND_TREE ? in.R * in.D : in.D;
    d.max_levels = in.max_levels;
    d.window = in.window;
    d.nstages = in.kind == SFFT_KIND_FFAST ? in.R : 0;
    d.max_peel_rounds = in.max_peel_rounds;
    d.found_cap = in.found_cap;
    d.multi_cap = in.multi_cap;
    d.col_rows = in.multi_cap;
    d.l1 = (in.kind == SFFT_KIND_TREE && !no_jump && in.l1_resolve) ? 1 : 0;
    d.jump_L = (in.kind == SFFT_KIND_TREE && !no_jump && !d.l1) ? in.jump_L : 0;
    d.mpp = in.mpp;
    d.precision = in.precision;
    d.fp16 = in.kind == SFFT_KIND_TREE && in.sample_format == SFFT_SAMPLES_F16 ? 1 : 0;
    d.col_key = -1;
    d.col_ltc = 0;
    d.col_dz = 0;
    d.l0_tile_lg = in.fft_tile_lg;
    d.enum_lane_blocks = in.kind == SFFT_KIND_TREE && in.enum_share > 0 ? in.enum_share : kEnumLaneBlocks;
    d.n_starts = in.kind == SFFT_KIND_FFAST ? in.peel_starts : 0;
    d.rf_iters = in.kind == SFFT_KIND_FFAST ? in.rf_iters : 0;
    d.rf_m = in.rf_m;
    for (int r = 0; r < SFFT_MAX_ROUNDS; r++) d.rf_off[r] = in.rf_off[r];
    for (int i = 0; i < SFFT_MAX_PEEL_STARTS; i++) d.start_f[i] = in.peel_start_f[i];
    for (int j = 0; j < SFFT_MAX_STAGES; j++) d.stageB[j] = in.stage_B[j];
    for (int j = 0; j <= SFFT_MAX_STAGES; j++) d.stageOff[j] = p->stage_off[j];
    for (int r = 0; r < SFFT_MAX_ROUNDS; r++) d.shift[r] = in.shift[r];
    d.eps0 = in.eps0;
    d.eps1 = in.eps1;
    d.zero_k = in.zero_k;
    d.single_k = in.single_k;
    d.noise_var = in.noise_var;
    d.noise_p_den = p->noise_p_den;
    d.noise_at = p->noise_at;
    d.y0_off = y0;
    d.found_off = fc;
    d.multi_off = mc;
    d.fst_off = fst;
    d.jc_off = jc;
    if (d.l1) {
      // rows of the column pass: the expected number of level-0 multi-tons
      // (K tones in B0 classes, Poisson: B0 (1 - e^-l (1 + l)), l = K / B0)
      // with half of it and 64 rows to spare; more open classes than that
      // leave the signal PARTIAL
      {
        const double lam = (double)in.K / (double)in.B0;
        const double ex = (double)in.B0 * (1.0 - std::exp(-lam) * (1.0 + lam));
        d.col_rows = (int32_t)std::min<int64_t>(d.multi_cap, (int64_t)std::ceil(1.5 * ex) + 64);
      }
      d.col_key = d.log2B0 + 32 * d.fp16 + (in.col_form == 2 ? 64 : in.col_form == 3 ? 128 : 0);
      d.col_ltc = in.col_form == 3 ? 4 : 14 - d.log2B0;  // 16 columns; else 512 / (B0 / 32)
      // classes open below depth col_dz go to the deep resolution (one L-point
      // FFT of the row, then L / 2^dd terms per sum instead of 2^dd): from about
      // half the depth of the tree, for rows an LDS transform holds
      const int lgL = d.log2N - d.log2B0;
      d.col_dz = lgL <= kLog2FftMax ? std::min(kColLaneDepth, (lgL + 1) / 2) : 0;
    }
    if (in.kind == SFFT_KIND_TREE) {
      y0 += (int64_t)d.n * in.B0;
      mc += d.multi_cap;
      if (d.l1) jc += (int64_t)d.col_rows * (in.N / in.B0);
      tree.push_back({(int64_t)d.n * in.B0 * (in.max_levels + 1), s});
      maxB0 = std::max<int64_t>(maxB0, in.B0);
    } else {
      y0 += (int64_t)in.D * p->nb;
      fst += p->nb * (2 * (int64_t)in.D + 2);
      ffast.push_back({(int64_t)in.D * p->nb, s});
      for (int j = 0; j < in.R; j++) maxStage = std::max<int64_t>(maxStage, in.stage_B[j]);
    }
    fc += d.found_cap;
    nmax = std::max(nmax, d.n);
    maxFcap = std::max(maxFcap, d.found_cap);
    Y.desc[s] = d;
  }
  for (int s = 0; s < nsig; s++)
    if (Y.desc[s].kind == SFFT_KIND_TREE && jump_level(Y.desc[s]) <= Y.desc[s].max_levels) Y.any_jump = true;
  for (int s = 0; s < nsig; s++)
    if (ps[s]->info.kind == SFFT_KIND_TREE) {
      Y.gather_u = ps[s]->info.gather_unroll;
      break;
    }
  // longest solves first (LPT order) for the persistent level-0 launches
  std::stable_sort(tree.begin(), tree.end(), [](auto &a, auto &b) { return a.first > b.first; });
  std::stable_sort(ffast.begin(), ffast.end(), [](auto &a, auto &b) { return a.first > b.first; });
  for (auto &t : tree) Y.lists.push_back(t.second);
  for (auto &t : ffast) Y.lists.push_back(t.second);
  // level-0 item prefixes over the tree list: rounds, and 256-class chunks
  Y.l0_at = Y.lists.size();
  int32_t acc0 = 0;
  for (auto &t : tree) {
    Y.lists.push_back(acc0);
    acc0 += Y.desc[t.second].R;
  }
  Y.lists.push_back(acc0);
  // level-0 classification: lanes per class.  The team enumeration is
  // compiled in where some noisy class's candidate range is longer than its
  // plan's enum_share blocks of 32; the classes are then spread over 2^lg
  // lanes (64 >> lg classes a wave), doubled up to kL0SpreadAuto while such
  // classes fill at most kL0SpreadWaves waves -- a small batch then
  // enumerates on every SIMD, each class by a team -- unless a plan fixes it
  {
    int64_t nclass = 0;
    int req = 0;
    for (auto &t : tree) {
      const SigDesc &d = Y.desc[t.second];
      req = std::max(req, ps[t.second]->info.l0_spread);
      if (d.mode != SFFT_NOISY) continue;
      const int64_t L0 = d.N >> d.log2B0;
      const int64_t cnt = (d.window > 0 && d.D >= 2 && 2 * (int64_t)d.window + 1 < L0) ? 2 * (int64_t)d.window + 1 : L0;
      if (((cnt + 31) >> 5) > d.enum_lane_blocks) {
        Y.any_noisy0 = 1;
        nclass += d.B0;
      }
    }
    int sp = req;
    if (sp == 0) {
      sp = 1;
      while (nclass > 0 && sp < kL0SpreadAuto && nclass * 2 * sp <= (int64_t)kL0SpreadWaves * 64) sp *= 2;
    }
    Y.l0_spread_lg = ilog2(sp);
    if (sp > 1) Y.any_noisy0 = 1;
  }
  Y.l0c_at = Y.lists.size();
  int32_t acc1 = 0;
  const int64_t per_item = kThreads >> Y.l0_spread_lg;
  for (auto &t : tree) {
    Y.lists.push_back(acc1);
    acc1 += (int32_t)((Y.desc[t.second].B0 + per_item - 1) / per_item);
  }
  Y.lists.push_back(acc1);
  Y.lists.push_back(0);
  Y.ntree = (int)tree.size();
  Y.nffast = (int)ffast.size();
  Y.l0_items = acc0;
  Y.l0c_items = acc1;
  Y.nmax = nmax;
  Y.max_B0 = maxB0;
  Y.max_stage = maxStage;
  Y.max_found_cap = (int)npow2(maxFcap);
  // dense-pass items: 4096 rows for batches of 64 signals or more, fewer
  // rows (more work-groups per signal) for smaller batches
  Y.jrows = kJumpItemRows;
  while (Y.jrows > kJumpItemRowsMin && (int64_t)Y.jrows * 64 > (int64_t)kJumpItemRows * nsig) Y.jrows >>= 1;
  for (int s = 0; s < nsig; s++) {
    const SigDesc &d = Y.desc[s];
    if (d.kind == SFFT_KIND_TREE && d.precision == 1) Y.any_fp32 = 1;
    if (d.kind == SFFT_KIND_TREE && d.mode == SFFT_NOISY && !(d.noise_var > 0.0)) Y.any_noise_est = 1;
    if (d.l1 && ps[s]->info.col_form == 2) Y.col16_mask |= d.fp16 ? 2 : 1;
    else if (d.l1 && ps[s]->info.col_form == 3) Y.col16_mask |= d.fp16 ? 8 : 4;
    else if (d.l1) (d.fp16 ? Y.col_f16_mask : Y.col_lp_mask) |= 1 << (d.log2B0 - 9);  // bit LP - 4, B0 = 2^(LP + 5)
    // the team enumeration below level 0 is compiled in only where some noisy
    // class has a candidate range longer than its plan's enum_share blocks
    if (d.kind == SFFT_KIND_TREE && d.mode == SFFT_NOISY) {
      const int64_t L0 = d.N >> d.log2B0;
      // the subtree levels' ranges: L0 / 2 candidates at level 1 (a window, if
      // any, is the same at every level)
      const int64_t cnt1 = (d.window > 0 && d.D >= 2 && 2 * (int64_t)d.window + 1 < L0 / 2) ? 2 * (int64_t)d.window + 1 : L0 / 2;
      if (d.max_levels >= 1 && ((cnt1 + 31) >> 5) > d.enum_lane_blocks) Y.any_noisy = 1;
    }
    if (d.kind == SFFT_KIND_TREE)
      Y.l0_lds = std::max<int32_t>(Y.l0_lds, (int32_t)(sizeof(float2) * (size_t)d.D << d.l0_tile_lg));
    if (d.kind == SFFT_KIND_TREE && d.jump_L >= (1 << kJumpMfmaMinLg)) Y.any_wide_jump = 1;
    if (d.l1 && d.col_dz > 0 && d.col_dz < d.max_levels)
      Y.deep_lds = std::max<int32_t>(Y.deep_lds, (int32_t)(sizeof(float2) << (d.log2N - d.log2B0)));
  }
  // arenas
  Y.n_y0 = y0;
  Y.n_fst = fst;
  Y.n_found = fc;
  Y.n_multi = mc;
  Y.n_mvec = mc * (int64_t)nmax;  // multi-ton vectors use the batch-wide stride nmax
  Y.n_jacc = Y.any_jump ? mc * (int64_t)kJumpMax : 0;
  Y.n_jcol = jc;
  const size_t ns = (size_t)nsig;
  size_t o = 0;
  auto part = [&](size_t &off, size_t bytes) {
    off = o;
    o = align_up(o + bytes);
  };
  part(Y.o_desc, sizeof(SigDesc) * ns);
  part(Y.o_io, sizeof(SigIO) * ns);
  part(Y.o_st, sizeof(SigState) * ns);
  part(Y.o_lists, sizeof(int32_t) * Y.lists.size());
  part(Y.o_pre, kPre * sizeof(int32_t) * (ns + 1));
  part(Y.o_out, (sizeof(int64_t) + sizeof(int32_t)) * 2);
  part(Y.o_y0, sizeof(float2) * (size_t)Y.n_y0);
  part(Y.o_fst, sizeof(double2) * (size_t)Y.n_fst);
  part(Y.o_ff, sizeof(int64_t) * (size_t)Y.n_found);
  part(Y.o_fa, sizeof(double2) * (size_t)Y.n_found);
  part(Y.o_mc, 2 * sizeof(int64_t) * (size_t)Y.n_multi);
  part(Y.o_my, 2 * sizeof(float2) * (size_t)Y.n_mvec);
  part(Y.o_mz, 2 * sizeof(double2) * (size_t)Y.n_mvec);
  part(Y.o_jacc, sizeof(double2) * (size_t)Y.n_jacc);
  part(Y.o_jcol, sizeof(float2) * (size_t)Y.n_jcol);
  // deep-resolution hand-off: a counter, then a list entry and a mask per multi-ton slot
  part(Y.o_deep, Y.deep_lds ? 256 + (sizeof(int2) + sizeof(uint64_t)) * (size_t)Y.n_multi : 0);
  Y.bytes = o;
  // static launch shape of every tree level: a signal gathers level by level
  // before its jump level, runs the dense pass and the subtree resolution at
  // it, and has no work after it
  int last = 0;
  for (int s = 0; s < nsig; s++) {
    const SigDesc &d = Y.desc[s];
    if (d.kind == SFFT_KIND_TREE)
      last = std::max(last, d.l1 ? 1 : std::min(d.max_levels, jump_level(d) + 1));
  }
  for (int l = 1; l <= last; l++) {
    LevelLaunch L{};
    int64_t nf = 0, nd = 0, nch = 0, nj = 0, nr = 0, ncol = 0, ncr = 0;
    for (int s = 0; s < nsig; s++) {
      const SigDesc &d = Y.desc[s];
      if (d.kind != SFFT_KIND_TREE || l > d.max_levels) continue;
      if (d.l1) {
        if (l == 1) {
          ncol += (((d.N >> d.log2B0) >> d.col_ltc) + kColItemAlign - 1) & ~(int64_t)(kColItemAlign - 1);
          ncr += d.multi_cap;
        }
        continue;
      }
      const int jl = jump_level(d);
      if (l > jl + 1) continue;
      const int64_t Bp = d.B0 << (l - 1);
      if (l >= jl) {  // the dense pass may run at jl (few classes) and runs at jl + 1
        nj += (Bp + Y.jrows - 1) / Y.jrows;
        nr += d.multi_cap;
      }
      if (l > jl) continue;
      const int64_t Bsmax = int64_t(1) << split_lg(d.D);
      if (Bp <= Bsmax) {
        nf += d.R;
      } else {
        nf += (int64_t)d.R * (Bp / Bsmax);
        nd += (int64_t)d.R * ((Bp + kChunk - 1) / kChunk);
      }
      nch += 2 * (int64_t)d.multi_cap;
    }
    L.fft = nf > 0;
    L.direct = nd > 0;
    L.children = nch > 0;
    L.jump = nj > 0;
    L.col = ncol > 0;
    // column pass: one resident work-group per CU (a multiple of 64, for the
    // XCD grouping of its items: 8 XCDs x up to 8 work-groups per segment)
    L.grid_col = (int)std::max<int64_t>(64, std::min<int64_t>((int64_t)ncu & ~63, ((ncol + 63) / 64) * 64));
    L.grid_col_resolve = (int)std::min<int64_t>(std::max<int64_t>((ncr + 64 / kColGroup - 1) / (64 / kColGroup), 1), 4096);
    L.grid_col_deep = (int)std::min<int64_t>(std::max<int64_t>(ncr, 1), 2 * (int64_t)ncu);
    L.grid_fft = (int)std::min<int64_t>(std::max<int64_t>(nf, 1), 4096);
    L.grid_direct = (int)std::min<int64_t>(std::max<int64_t>(nd, 1), 8192);
    L.grid_children = (int)std::min<int64_t>(std::max<int64_t>((nch + kThreads - 1) / kThreads, 1), 2048);
    L.grid_jump = (int)std::min<int64_t>(std::max<int64_t>(nj, 1), 8192);
    L.grid_resolve = (int)std::min<int64_t>(std::max<int64_t>(nr, 1), 4096);
    Y.levels.push_back(L);
  }
  return SFFT_OK;
}

// Launch context of a layout placed at `base` (a device slab of Y.bytes whose
// descriptor and list parts hold Y.desc and Y.lists).
void bind_layout(const Layout &Y, char *base, const float2 *tw, LaunchCtx &c) {
  c = LaunchCtx{};
  c.desc = (const SigDesc *)(base + Y.o_desc);
  c.io = nullptr;
  c.st = (SigState *)(base + Y.o_st);
  c.A.y0 = (float2 *)(base + Y.o_y0);
  c.A.fst = (double2 *)(base + Y.o_fst);
  c.A.found_f = (int64_t *)(base + Y.o_ff);
  c.A.found_a = (double2 *)(base + Y.o_fa);
  c.A.multi_c[0] = (int64_t *)(base + Y.o_mc);
  c.A.multi_c[1] = (int64_t *)(base + Y.o_mc) + Y.n_multi;
  c.A.multi_y[0] = (float2 *)(base + Y.o_my);
  c.A.multi_y[1] = (float2 *)(base + Y.o_my) + Y.n_mvec;
  c.A.multi_z[0] = (double2 *)(base + Y.o_mz);
  c.A.multi_z[1] = (double2 *)(base + Y.o_mz) + Y.n_mvec;
  c.A.pre = (int32_t *)(base + Y.o_pre);
  c.A.jacc = (double2 *)(base + Y.o_jacc);
  c.A.jcol = (float2 *)(base + Y.o_jcol);
  c.A.deep_count = (int32_t *)(base + Y.o_deep);
  c.A.deep_list = (int2 *)(base + Y.o_deep + 256);
  c.A.deep_mask = (uint64_t *)(base + Y.o_deep + 256 + sizeof(int2) * (size_t)Y.n_multi);
  c.deep_lds = Y.deep_lds;
  c.A.tw = tw;
  const int32_t *lists = (const int32_t *)(base + Y.o_lists);
  c.tree_list = lists;
  c.ffast_list = lists + Y.ntree;
  c.l0_pre = lists + Y.l0_at;
  c.l0c_pre = lists + Y.l0c_at;
  c.l0_items = Y.l0_items;
  c.l0c_items = Y.l0c_items;
  c.jstride = kJumpMax;
  c.jrows = Y.jrows;
  c.any_fp32 = Y.any_fp32;
  c.col_lp_mask = Y.col_lp_mask;
  c.col_f16_mask = Y.col_f16_mask;
  c.col16_mask = Y.col16_mask;
  c.any_noisy0 = Y.any_noisy0;
  c.l0_spread_lg = Y.l0_spread_lg;
  c.any_noisy = Y.any_noisy;
  c.any_noise_est = Y.any_noise_est;
  c.gather_u = Y.gather_u;
  c.l0_lds = Y.l0_lds;
  c.any_wide_jump = Y.any_wide_jump;
  c.nsig = (int32_t)Y.desc.size();
  c.ntree = Y.ntree;
  c.nffast = Y.nffast;
  c.nmax = Y.nmax;
  c.max_B0 = Y.max_B0;
  c.max_stage_B = Y.max_stage;
  c.max_found_cap = Y.max_found_cap;
}

int device_cus(int device) {
  int ncu = 256;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu < 16) {
    (void)hipGetLastError();
    ncu = 256;
  }
  return ncu;
}

// The whole pipeline of a layout bound in c, on stream s.  With `prof`, a
// timing event is recorded after every launch.
hipError_t launch_pipeline(const Layout &lay, const LaunchCtx &c, hipStream_t s, Prof *prof) {
  hipError_t e;
  auto mark = [&](int id) -> hipError_t {
    if (!prof) return hipSuccess;
    hipEvent_t ev;
    hipError_t r = hipEventCreate(&ev);
    if (r != hipSuccess) return r;
    prof->ev.push_back(ev);
    prof->id.push_back(id);
    return hipEventRecord(ev, s);
  };
  if ((e = mark(-1)) != hipSuccess) return e;
  if ((e = launch_reset(c, s)) != hipSuccess || (e = mark(SFFT_KERNEL_RESET)) != hipSuccess) return e;
  if ((e = launch_level0(c, s)) != hipSuccess || (e = mark(SFFT_KERNEL_LEVEL0)) != hipSuccess) return e;
  for (size_t i = 0; i < lay.levels.size(); i++) {
    const LevelLaunch &L = lay.levels[i];
    const int l = (int)i + 1;
    if ((e = launch_sched(c, l, s)) != hipSuccess || (e = mark(SFFT_KERNEL_SCHED)) != hipSuccess) return e;
    if (L.fft && ((e = launch_expand_fft(c, l, L.grid_fft, s)) != hipSuccess ||
                  (e = mark(SFFT_KERNEL_EXPAND_FFT | (l << 8))) != hipSuccess))
      return e;
    if (L.direct && ((e = launch_expand_direct(c, l, L.grid_direct, s)) != hipSuccess ||
                     (e = mark(SFFT_KERNEL_EXPAND_DIRECT | (l << 8))) != hipSuccess))
      return e;
    if (L.children && ((e = launch_children(c, l, L.grid_children, s)) != hipSuccess ||
                       (e = mark(SFFT_KERNEL_CHILDREN | (l << 8))) != hipSuccess))
      return e;
    if (L.jump && ((e = launch_jump_pass(c, l, L.grid_jump, s)) != hipSuccess ||
                   (e = mark(SFFT_KERNEL_JUMP_PASS | (l << 8))) != hipSuccess ||
                   (e = launch_jump_resolve(c, l, L.grid_resolve, s)) != hipSuccess ||
                   (e = mark(SFFT_KERNEL_JUMP_RESOLVE | (l << 8))) != hipSuccess))
      return e;
    if (L.col && ((e = launch_col_pass(c, L.grid_col, s)) != hipSuccess ||
                  (e = mark(SFFT_KERNEL_COL_PASS | (l << 8))) != hipSuccess ||
                  (e = launch_col_resolve(c, L.grid_col_resolve, s)) != hipSuccess ||
                  (e = mark(SFFT_KERNEL_COL_RESOLVE | (l << 8))) != hipSuccess))
      return e;
    if (L.col && c.deep_lds &&
        ((e = launch_col_deep(c, L.grid_col_deep, s)) != hipSuccess ||
         (e = mark(SFFT_KERNEL_COL_DEEP | (l << 8))) != hipSuccess))
      return e;
  }
  if ((e = launch_finalize(c, s)) != hipSuccess) return e;
  return mark(SFFT_KERNEL_FINALIZE);
}

bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

int32_t set_last_error(int32_t code) { return fail(code); }

}  // namespace sfft

namespace {

struct BatchCtx {
  int device = -1;
  std::vector<const sfft_plan_s *> plans;
  int nsig = 0;
  Layout lay;
  DevBuf slab;
  char *base = nullptr;
  LaunchCtx lc{};
  std::vector<SigIO> io_last;
  SigIO *io_pinned = nullptr;
  hipStream_t stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_io = nullptr;
  bool io_pending = false;

  ~BatchCtx() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (stream) (void)hipStreamDestroy(stream);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (ev_io) (void)hipEventDestroy(ev_io);
    if (io_pinned) (void)hipHostFree(io_pinned);
  }
  SigIO *io_dev() const { return (SigIO *)(base + lay.o_io); }
  SigState *st_dev() const { return (SigState *)(base + lay.o_st); }
  int64_t *count_dev() const { return (int64_t *)(base + lay.o_out); }
  int32_t *status_dev() const { return (int32_t *)((int64_t *)(base + lay.o_out) + 2); }

  int32_t build(const std::vector<const sfft_plan_s *> &ps, bool no_jump = false) {
    plans = ps;
    nsig = (int)ps.size();
    if (hipGetDevice(&device) != hipSuccess) return SFFT_EDEVICE;
    int32_t rc = make_layout(ps, no_jump, device_cus(device), lay);
    if (rc != SFFT_OK) return rc;
    if (slab.alloc(lay.bytes) != hipSuccess) return SFFT_ENOMEM;
    base = (char *)slab.p;
    if (hipMemcpy(base + lay.o_desc, lay.desc.data(), sizeof(SigDesc) * lay.desc.size(),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + lay.o_lists, lay.lists.data(), sizeof(int32_t) * lay.lists.size(),
                  hipMemcpyHostToDevice) != hipSuccess)
      return SFFT_EDEVICE;
    const float2 *tw = nullptr;
    if (device_twiddles(device, &tw) != hipSuccess) return SFFT_EDEVICE;
    bind_layout(lay, base, tw, lc);
    io_last.assign((size_t)nsig, SigIO{});
    return SFFT_OK;
  }
  hipError_t launch_all(const LaunchCtx &c, hipStream_t s, Prof *prof = nullptr) {
    return launch_pipeline(lay, c, s, prof);
  }
};

std::mutex g_batch_mu;
std::map<std::vector<const sfft_plan_s *>, std::unique_ptr<BatchCtx>> g_batches;

// drop every cached batch that uses plan p
void forget_plan(const sfft_plan_s *p) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (auto it = g_batches.begin(); it != g_batches.end();) {
    if (std::find(it->first.begin(), it->first.end(), p) != it->first.end()) it = g_batches.erase(it);
    else ++it;
  }
}

int32_t validate_and_fill(const sfft_params_t *pp, sfft_plan_s *pl) {
  const sfft_params_t &p = *pp;
  sfft_plan_info_t &in = pl->info;
  memset(&in, 0, sizeof(in));
  if (p.N < 2 || p.N > kMaxN || p.K < 1 || p.K > p.N || p.K > 4096) return SFFT_EINVAL;
  // the R-FFAST delay set replaces the D consecutive delays
  int32_t delays = p.delays;
  if (p.rf_iters != 0) {
    if (pow2(p.N) && p.nstage_B == 0) return SFFT_EUNSUPPORTED;
    if (p.rf_iters < 1 || p.rf_iters > SFFT_MAX_ROUNDS || p.rf_m < 2 ||
        (int64_t)p.rf_iters * p.rf_m > kMaxMeas)
      return SFFT_EINVAL;
    delays = p.rf_iters * p.rf_m;
  }
  if (delays < 1 || p.stages < 1) return SFFT_EINVAL;
  if (p.mode != SFFT_EXACT && p.mode != SFFT_NOISY) return SFFT_EINVAL;
  if (p.mode == SFFT_EXACT && delays < 2) return SFFT_EINVAL;
  if (p.window < 0) return SFFT_EINVAL;
  in.N = p.N;
  in.K = p.K;
  in.mode = p.mode;
  in.D = delays;
  in.window = p.window;
  in.eps0 = p.eps0;
  in.eps1 = p.eps1;
  in.zero_k = p.zero_k;
  in.single_k = p.single_k;
  in.noise_var = p.noise_var;
  in.max_peel_rounds = p.max_peel_rounds > 0 ? p.max_peel_rounds : 64;
  if (p.jump_L < 0 || p.jump_L > kJumpMax || (p.jump_L > 0 && !pow2(p.jump_L))) return SFFT_EINVAL;
  in.jump_L = p.jump_L;
  if (p.mpp != 0 && p.mpp != 2) return SFFT_EINVAL;
  in.mpp = p.mpp;
  if (p.precision != 0 && p.precision != 1) return SFFT_EINVAL;
  in.precision = p.precision;
  if (p.l1_resolve != 0 && p.l1_resolve != 1) return SFFT_EINVAL;
  if (p.sample_format != SFFT_SAMPLES_C64 && p.sample_format != SFFT_SAMPLES_F16) return SFFT_EINVAL;
  in.sample_format = p.sample_format;
  if (p.gather_unroll != 0 && p.gather_unroll != 2 && p.gather_unroll != 4 && p.gather_unroll != 8)
    return SFFT_EINVAL;
  in.gather_unroll = p.gather_unroll ? p.gather_unroll : 4;
  in.found_cap = (int32_t)std::max<int64_t>(64, npow2(2 * p.K));
  in.multi_cap = (int32_t)std::max<int64_t>(64, p.K);
  memset(pl->stage_off, 0, sizeof(pl->stage_off));
  double phi = 1.0;
  int64_t cnt = 0;
  if (pow2(p.N) && p.nstage_B == 0) {
    // binary tree search over R rounds sharing B0
    if (p.stages > SFFT_MAX_ROUNDS) return SFFT_EINVAL;
    if ((int64_t)p.stages * delays > kMaxMeas) return SFFT_EUNSUPPORTED;
    if (delays > kMaxD) return SFFT_EUNSUPPORTED;
    int64_t B0 = p.B0;
    if (B0 <= 0) B0 = std::min<int64_t>(npow2(2 * p.K), p.N);
    if (!pow2(B0) || B0 > p.N) return SFFT_EINVAL;
    if (B0 > kFftMax) return SFFT_EUNSUPPORTED;
    {
      const int top = std::min(ilog2(B0), split_lg(delays));
      if (p.fft_tile_lg != 0 && (p.fft_tile_lg < 5 || p.fft_tile_lg > top)) return SFFT_EINVAL;
      in.fft_tile_lg = p.fft_tile_lg ? p.fft_tile_lg : top;
    }
    if (p.peel_starts != 0) return SFFT_EUNSUPPORTED;
    if (p.mpp == 2 && p.mode != SFFT_EXACT) return SFFT_EUNSUPPORTED;
    if (p.mpp == 2 && (int64_t)p.stages * (delays - 2) < 2) return SFFT_EINVAL;
    in.kind = SFFT_KIND_TREE;
    in.R = p.stages;
    in.B0 = B0;
    const int full = ilog2(p.N / B0);
    in.max_levels = (p.max_levels < 0 || p.max_levels > full) ? full : p.max_levels;
    // level-1 column pass: B0 = 32 P with P = 16 ... 256, at least 32768 / B0
    // and 16 columns
    in.l1_resolve = p.l1_resolve && (B0 == 512 || B0 == 1024 || B0 == 2048 || B0 == 4096 || B0 == 8192) &&
                    p.N / B0 >= std::max<int64_t>(32768 / B0, 16) && in.max_levels >= 1;
    if (p.col_form < 0 || p.col_form > 3 || (p.col_form >= 2 && B0 != 2048)) return SFFT_EINVAL;
    if (p.enum_share < 0 || p.enum_share > kEnumLaneBlocks) return SFFT_EINVAL;
    in.enum_share = p.enum_share ? p.enum_share : kEnumShareDefault;
    if (p.l0_spread < 0 || p.l0_spread > kL0SpreadMax || (p.l0_spread & (p.l0_spread - 1))) return SFFT_EINVAL;
    in.l0_spread = p.l0_spread;
    // the library's choice: the 16-column form at B0 = 2048, the 32-row form elsewhere
    in.col_form = in.l1_resolve ? (p.col_form > 0 ? p.col_form : (B0 == 2048 ? 3 : 1)) : 0;
    SplitMix64 g{p.seed};
    for (int r = 0; r < p.stages; r++) {
      if (r == 0 && p.identity_round0) {
        in.sigma[r] = 1;
        in.shift[r] = 0;
      } else {
        const uint64_t a = g.next(), b = g.next();
        in.sigma[r] = 2 * (a % (uint64_t)(p.N / 2)) + 1;
        in.shift[r] = b % (uint64_t)p.N;
      }
    }
    phi = std::pow(1.0 - 1.0 / (double)B0, (double)p.K);
    cnt = (int64_t)p.stages * delays * B0;
  } else {
    // FFAST: co-prime stages, from explicit sizes or the prime powers of N
    std::vector<int64_t> st;
    if (p.nstage_B > 0) {
      if (p.nstage_B > SFFT_MAX_STAGES) return SFFT_EINVAL;
      int64_t prod = 1;
      for (int j = 0; j < p.nstage_B; j++) {
        const int64_t b = p.stage_B[j];
        if (b < 1 || p.N % b) return SFFT_EINVAL;
        for (int64_t o : st)
          if (gcd64((uint64_t)o, (uint64_t)b) != 1) return SFFT_EINVAL;
        st.push_back(b);
        prod *= b;
      }
      (void)prod;
    } else {
      int64_t rest = p.N;
      for (int64_t q = 2; q * q <= rest; q++) {
        if (rest % q) continue;
        int64_t pw = 1;
        while (rest % q == 0) {
          rest /= q;
          pw *= q;
        }
        st.push_back(pw);
      }
      if (rest > 1) st.push_back(rest);
      if ((int)st.size() != p.stages) return SFFT_EUNSUPPORTED;
    }
    if ((int)st.size() > SFFT_MAX_STAGES) return SFFT_EUNSUPPORTED;
    if (p.mpp != 0 || p.precision != 0 || p.sample_format != SFFT_SAMPLES_C64) return SFFT_EUNSUPPORTED;
    SplitMix64 g{p.seed};
    in.rf_iters = p.rf_iters;
    in.rf_m = p.rf_iters ? p.rf_m : 0;
    for (int c = 0; c < p.rf_iters; c++) in.rf_off[c] = g.next() % (uint64_t)p.N;
    if (p.peel_starts < 0 || p.peel_starts > SFFT_MAX_PEEL_STARTS) return SFFT_EINVAL;
    in.peel_starts = p.peel_starts;
    if (p.peel_starts > 0) {
      int given = 0;
      for (int i = 0; i < p.peel_starts; i++) {
        if (p.peel_start_f[i] >= p.N) return SFFT_EINVAL;
        given += p.peel_start_f[i] >= 0;
      }
      if (given != 0 && given != p.peel_starts) return SFFT_EINVAL;
      for (int i = 0; i < p.peel_starts; i++)
        in.peel_start_f[i] = given ? p.peel_start_f[i] : (int64_t)(g.next() % (uint64_t)p.N);
    }
    if (delays > kMaxMeas || p.N >= (int64_t(1) << 31)) return SFFT_EUNSUPPORTED;
    in.kind = SFFT_KIND_FFAST;
    in.R = (int32_t)st.size();
    int64_t off = 0;
    double wphi = 0;
    for (size_t j = 0; j < st.size(); j++) {
      const int64_t b = st[j];
      if (pow2(b) ? b > kFftMax : b > kDirectMax) return SFFT_EUNSUPPORTED;
      in.stage_B[j] = b;
      in.sigma[j] = 1;
      in.shift[j] = 0;
      pl->stage_off[j] = off;
      off += b;
      wphi += (double)b * std::pow(1.0 - 1.0 / (double)b, (double)p.K);
    }
    for (size_t j = st.size(); j <= SFFT_MAX_STAGES; j++) pl->stage_off[j] = off;
    if (off > kMaxFfastBuckets) return SFFT_EUNSUPPORTED;
    pl->nb = off;
    phi = wphi / (double)off;
    cnt = off * delays;
  }
  // noise estimator constants: p-quantile of B |yhat|^2 with p = min(1/4, phi/2)
  const double q = std::min(0.25, phi / 2.0);
  pl->noise_at = (int64_t)(q * (double)(cnt - 1));
  pl->noise_p_den = -std::log(1.0 - q / phi);
  return SFFT_OK;
}

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

int32_t check_io(const void *x, const void *idx, const void *val) {
  if (!is_device_ptr(x) || !is_device_ptr(idx) || !is_device_ptr(val)) return SFFT_EINVAL;
  return SFFT_OK;
}

BatchCtx *single_ctx(sfft_plan_t plan, int32_t *rc) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    *rc = SFFT_EDEVICE;
    return nullptr;
  }
  if (!plan->single || plan->single->device != dev) {
    plan->single.reset(new BatchCtx());
    const int32_t r = plan->single->build({plan});
    if (r != SFFT_OK) {
      plan->single.reset();
      *rc = r;
      return nullptr;
    }
  }
  *rc = SFFT_OK;
  return plan->single.get();
}

int32_t run_single(sfft_plan_t plan, const void *x, int64_t *out_idx, void *out_val,
                   int64_t *d_count, int32_t *d_status, hipStream_t stream) {
  int32_t rc;
  BatchCtx *b = single_ctx(plan, &rc);
  if (!b) return rc;
  LaunchCtx c = b->lc;
  c.io = nullptr;
  c.io1.x = (const float2 *)x;
  c.io1.idx = out_idx;
  c.io1.val = (float2 *)out_val;
  c.io1.count = d_count ? d_count : b->count_dev();
  c.io1.status = d_status ? d_status : b->status_dev();
  if (b->launch_all(c, stream) != hipSuccess) return SFFT_EDEVICE;
  return SFFT_OK;
}

// ------------------------------------------------------- host-gather solves
// A host-resident signal is solved with only the samples each step reads
// crossing to the device: the host packs them in (round or stage, m, delay)
// order, k_scatter writes them to their positions in a device image of x,
// and the usual kernels run on that image (the dense pass, which reads all
// of x, is switched off).  Tree levels are decided one at a time: after a
// level's scheduling the host reads whether the next level has open classes.
// A fixed set of worker threads that split an index range [0, n) between
// them and the calling thread; kept for the life of a host-gather context.
struct GatherPool {
  std::vector<std::thread> th;
  std::mutex mu;
  std::condition_variable cv, done;
  std::function<void(int64_t, int64_t)> job;
  int64_t n = 0;
  uint64_t gen = 0;
  int pending = 0;
  bool stop = false;
  int parts = 1;
  explicit GatherPool(int workers) : parts(workers + 1) {
    for (int w = 0; w < workers; w++) th.emplace_back([this, w] { loop(w + 1); });
  }
  ~GatherPool() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    for (auto &t : th) t.join();
  }
  void loop(int part) {
    uint64_t seen = 0;
    for (;;) {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || gen != seen; });
      if (stop) return;
      seen = gen;
      const int64_t a = n * part / parts, b = n * (part + 1) / parts;
      lk.unlock();
      job(a, b);
      lk.lock();
      if (--pending == 0) done.notify_one();
    }
  }
  void run(int64_t count, const std::function<void(int64_t, int64_t)> &f) {
    {
      std::lock_guard<std::mutex> lk(mu);
      job = f;
      n = count;
      pending = (int)th.size();
      gen++;
    }
    cv.notify_all();
    f(0, count / parts);
    std::unique_lock<std::mutex> lk(mu);
    done.wait(lk, [&] { return pending == 0; });
  }
};

struct HostCtx {
  int device = -1;
  BatchCtx b;
  std::unique_ptr<GatherPool> pool;
  DevBuf img, packed, res;
  float2 *staging = nullptr;   // pinned host buffer of `cap` samples
  uint64_t *word = nullptr;    // pinned host word for the level mask
  size_t cap = 0;
  hipStream_t stream = nullptr;
  ~HostCtx() {
    if (staging) (void)hipHostFree(staging);
    if (word) (void)hipHostFree(word);
    if (stream) (void)hipStreamDestroy(stream);
  }
  int32_t reserve(size_t n) {
    if (n <= cap) return SFFT_OK;
    if (staging) (void)hipHostFree(staging);
    staging = nullptr;
    cap = 0;
    if (hipHostMalloc((void **)&staging, n * sizeof(float2), 0) != hipSuccess) return SFFT_ENOMEM;
    if (packed.alloc(n * sizeof(float2)) != hipSuccess) return SFFT_ENOMEM;
    cap = n;
    return SFFT_OK;
  }
};

// samples read by tree level `level` (FFAST: its stages, level 0)
int64_t level_samples(const sfft_plan_s *p, int level) {
  const sfft_plan_info_t &in = p->info;
  if (in.kind == SFFT_KIND_FFAST) return p->nb * in.D;
  const int64_t Bp = level == 0 ? in.B0 : (in.B0 << (level - 1));
  return (int64_t)in.R * in.D * Bp;
}

// position in x of packed sample i of `level` (the order k_scatter writes)
inline uint64_t sample_pos(const sfft_plan_s *p, int level, int lgB0, int64_t i) {
  const sfft_plan_info_t &in = p->info;
  const uint64_t N = (uint64_t)in.N;
  const int dl = (int)(i % in.D);
  const int64_t rm = i / in.D;
  if (in.kind == SFFT_KIND_FFAST) {
    int j = 0;
    while (j + 1 < in.R && p->stage_off[j + 1] <= rm) j++;
    const uint64_t m = (uint64_t)(rm - p->stage_off[j]);
    uint64_t tau = (uint64_t)dl;
    if (in.rf_iters > 0) {
      const int c = dl / in.rf_m, t = dl % in.rf_m;
      tau = (in.rf_off[c] + ((uint64_t)t << c)) % N;
    }
    return (m * (N / (uint64_t)in.stage_B[j]) + tau) % N;
  }
  const int lb = lgB0 + (level > 0 ? level - 1 : 0);
  const uint64_t Bp = (uint64_t)1 << lb, Lp = N >> lb;
  const int r = (int)(rm >> lb);
  const uint64_t m = (uint64_t)rm & (Bp - 1);
  return (m * Lp + (level > 0 ? (Lp >> 1) : 0) + in.shift[r] + (uint64_t)dl) & (N - 1);
}

void gather_samples(const sfft_plan_s *p, int level, const float2 *x, float2 *out, int64_t n,
                    GatherPool *pool) {
  const int lgB0 = p->info.kind == SFFT_KIND_TREE ? ilog2(p->info.B0) : 0;
  auto work = [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; i++) out[i] = x[sample_pos(p, level, lgB0, i)];
  };
  if (!pool || n < (int64_t(1) << 13)) {
    work(0, n);
    return;
  }
  pool->run(n, work);
}

HostCtx *host_ctx(sfft_plan_t plan, int32_t *rc) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    *rc = SFFT_EDEVICE;
    return nullptr;
  }
  if (!plan->host || plan->host->device != dev) {
    std::unique_ptr<HostCtx> h(new HostCtx());
    h->device = dev;
    const unsigned hw = std::thread::hardware_concurrency();
    const int workers = (int)std::min(15u, hw > 1 ? hw - 1 : 0u);
    if (workers > 0) h->pool.reset(new GatherPool(workers));
    int32_t r = h->b.build({plan}, /*no_jump=*/true);
    const int64_t K = plan->info.K;
    if (r == SFFT_OK &&
        (h->img.alloc(sizeof(float2) * (size_t)plan->info.N) != hipSuccess ||
         h->res.alloc((sizeof(int64_t) + sizeof(float2)) * (size_t)K + 16) != hipSuccess ||
         hipHostMalloc((void **)&h->word, sizeof(uint64_t), 0) != hipSuccess))
      r = SFFT_ENOMEM;
    if (r == SFFT_OK && (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess ||
                         hipMemsetAsync(h->img.p, 0, sizeof(float2) * (size_t)plan->info.N, h->stream) !=
                             hipSuccess))
      r = SFFT_EDEVICE;
    if (r != SFFT_OK) {
      *rc = r;
      return nullptr;
    }
    plan->host = std::move(h);
  }
  *rc = SFFT_OK;
  return plan->host.get();
}

}  // namespace

// ================================================================== C-ABI
extern "C" {

void sfft_params_init(sfft_params_t *p, int64_t N, int64_t K, int32_t stages, int32_t delays,
                      uint64_t seed) {
  memset(p, 0, sizeof(*p));
  p->N = N;
  p->K = K;
  p->stages = stages;
  p->delays = delays;
  p->seed = seed;
  p->mode = SFFT_EXACT;
  p->B0 = 0;
  p->max_levels = -1;
  p->window = 0;
  p->identity_round0 = 0;
  p->nstage_B = 0;
  p->max_peel_rounds = 64;
  p->jump_L = 128;
  p->eps0 = 1e-4;
  p->eps1 = 1e-4;
  p->zero_k = 4.0;
  p->single_k = 4.0;
  p->noise_var = 0.0;
  p->mpp = 0;
  p->precision = 0;
  p->rf_iters = 0;
  p->rf_m = 0;
  p->peel_starts = 0;
  for (int i = 0; i < SFFT_MAX_PEEL_STARTS; i++) p->peel_start_f[i] = -1;
  p->l1_resolve = 1;
}

sfft_plan_t sfft_plan_ex(const sfft_params_t *p) {
  if (!p) {
    fail(SFFT_EINVAL);
    return nullptr;
  }
  std::unique_ptr<sfft_plan_s> pl(new sfft_plan_s());
  const int32_t rc = validate_and_fill(p, pl.get());
  if (rc != SFFT_OK) {
    fail(rc);
    return nullptr;
  }
  g_last_error = SFFT_OK;
  return pl.release();
}

sfft_plan_t sfft_plan(int64_t N, int64_t K, int32_t stages, int32_t delays, uint64_t seed) {
  sfft_params_t p;
  sfft_params_init(&p, N, K, stages, delays, seed);
  return sfft_plan_ex(&p);
}

int32_t sfft_plan_info(sfft_plan_t plan, sfft_plan_info_t *out) {
  if (!plan || !out) return fail(SFFT_EINVAL);
  *out = plan->info;
  return SFFT_OK;
}

void sfft_destroy(sfft_plan_t plan) {
  if (!plan) return;
  forget_plan(plan);
  delete plan;
}

int64_t sfft_exec(sfft_plan_t plan, const void *x, int64_t *out_idx, void *out_val) {
  if (!plan) return fail(SFFT_EINVAL);
  int32_t rc = check_io(x, out_idx, out_val);
  if (rc != SFFT_OK) return fail(rc);
  rc = run_single(plan, x, out_idx, out_val, nullptr, nullptr, nullptr);
  if (rc != SFFT_OK) return fail(rc);
  int64_t cnt = 0;
  if (hipMemcpy(&cnt, plan->single->count_dev(), sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(SFFT_EDEVICE);
  return cnt;
}

int32_t sfft_exec_async(sfft_plan_t plan, const void *x, int64_t *out_idx, void *out_val,
                        int64_t *d_count, int32_t *d_status, void *stream) {
  if (!plan) return fail(SFFT_EINVAL);
  int32_t rc = check_io(x, out_idx, out_val);
  if (rc != SFFT_OK) return fail(rc);
  if ((d_count && !is_device_ptr(d_count)) || (d_status && !is_device_ptr(d_status)))
    return fail(SFFT_EINVAL);
  rc = run_single(plan, x, out_idx, out_val, d_count, d_status, as_stream(stream));
  return rc == SFFT_OK ? SFFT_OK : fail(rc);
}

int32_t sfft_exec_noalloc(sfft_plan_t plan, const void *x, int64_t *out_idx, void *out_val,
                          int64_t *d_count, int32_t *d_status, void *stream) {
  if (!plan) return fail(SFFT_EINVAL);
  int32_t rc = check_io(x, out_idx, out_val);
  if (rc != SFFT_OK) return fail(rc);
  if (!is_device_ptr(d_count) || !is_device_ptr(d_status)) return fail(SFFT_EINVAL);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SFFT_EDEVICE);
  char *base = nullptr;
  if (noalloc_scratch(dev, &base) != hipSuccess) return fail(SFFT_EDEVICE);
  if (!plan->na_lay || plan->na_dev != dev) {
    std::unique_ptr<Layout> Y(new Layout());
    rc = make_layout({plan}, false, device_cus(dev), *Y);
    if (rc != SFFT_OK) return fail(rc);
    plan->na_lay = std::move(Y);
    plan->na_dev = dev;
  }
  const Layout &Y = *plan->na_lay;
  if (kNoAllocTwBytes + Y.bytes > kNoAllocScratchBytes) return fail(SFFT_ETOOBIG);
  char *slab = base + kNoAllocTwBytes;
  const hipStream_t s = as_stream(stream);
  if (hipMemcpyAsync(slab + Y.o_desc, Y.desc.data(), sizeof(SigDesc) * Y.desc.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(slab + Y.o_lists, Y.lists.data(), sizeof(int32_t) * Y.lists.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(SFFT_EDEVICE);
  LaunchCtx c;
  bind_layout(Y, slab, (const float2 *)base, c);
  c.io1.x = (const float2 *)x;
  c.io1.idx = out_idx;
  c.io1.val = (float2 *)out_val;
  c.io1.count = d_count;
  c.io1.status = d_status;
  if (launch_pipeline(Y, c, s, nullptr) != hipSuccess) return fail(SFFT_EDEVICE);
  return SFFT_OK;
}

int32_t sfft_exec_batch_ex(const sfft_plan_t *plans, const void *const *xs, int64_t *const *idx,
                           void *const *vals, int64_t *d_counts, int32_t *d_status, int32_t n,
                           void *stream, int32_t flags) {
  if (!plans || !xs || !idx || !vals || n < 1) return fail(SFFT_EINVAL);
  if (!is_device_ptr(d_counts) || !is_device_ptr(d_status)) return fail(SFFT_EINVAL);
  std::vector<const sfft_plan_s *> key(plans, plans + n);
  for (int i = 0; i < n; i++) {
    if (!plans[i]) return fail(SFFT_EINVAL);
    const int32_t rc = check_io(xs[i], idx[i], vals[i]);
    if (rc != SFFT_OK) return fail(rc);
  }
  std::lock_guard<std::mutex> lk(g_batch_mu);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SFFT_EDEVICE);
  auto &slot = g_batches[key];
  if (!slot || slot->device != dev) {
    slot.reset(new BatchCtx());
    const int32_t rc = slot->build(key);
    if (rc != SFFT_OK) {
      g_batches.erase(key);
      return fail(rc);
    }
    if (hipStreamCreateWithFlags(&slot->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&slot->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&slot->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&slot->ev_io, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&slot->io_pinned, sizeof(SigIO) * (size_t)n) != hipSuccess) {
      g_batches.erase(key);
      return fail(SFFT_EDEVICE);
    }
  }
  BatchCtx *b = slot.get();
  hipStream_t caller = as_stream(stream);
  // per-call pointers: upload only when they changed
  std::vector<SigIO> io(n);
  for (int i = 0; i < n; i++) {
    io[i] = SigIO{};
    io[i].x = (const float2 *)xs[i];
    io[i].idx = idx[i];
    io[i].val = (float2 *)vals[i];
    io[i].count = d_counts + i;
    io[i].status = d_status + i;
  }
  if (hipEventRecord(b->ev_in, caller) != hipSuccess ||
      hipStreamWaitEvent(b->stream, b->ev_in, 0) != hipSuccess)
    return fail(SFFT_EDEVICE);
  if (memcmp(io.data(), b->io_last.data(), sizeof(SigIO) * (size_t)n) != 0) {
    if (b->io_pending && hipEventSynchronize(b->ev_io) != hipSuccess) return fail(SFFT_EDEVICE);
    memcpy(b->io_pinned, io.data(), sizeof(SigIO) * (size_t)n);
    if (hipMemcpyAsync(b->io_dev(), b->io_pinned, sizeof(SigIO) * (size_t)n, hipMemcpyHostToDevice,
                       b->stream) != hipSuccess ||
        hipEventRecord(b->ev_io, b->stream) != hipSuccess)
      return fail(SFFT_EDEVICE);
    b->io_pending = true;
    b->io_last = io;
  }
  LaunchCtx c = b->lc;
  c.io = b->io_dev();
  if (flags & kBatchPrepareOnly) {
    // nothing launched: the caller runs the pipeline on the batch's stream
  } else if (flags & SFFT_BATCH_NO_GRAPH) {
    if (b->launch_all(c, b->stream) != hipSuccess) return fail(SFFT_EDEVICE);
  } else {
    if (!b->gexec) {
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(SFFT_EDEVICE);
      const hipError_t le = b->launch_all(c, b->stream);
      const hipError_t ce = hipStreamEndCapture(b->stream, &g);
      if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(SFFT_EDEVICE);
      }
      const hipError_t ie = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        b->gexec = nullptr;
        return fail(SFFT_EDEVICE);
      }
    }
    if (hipGraphLaunch(b->gexec, b->stream) != hipSuccess) return fail(SFFT_EDEVICE);
  }
  if (hipEventRecord(b->ev_out, b->stream) != hipSuccess ||
      hipStreamWaitEvent(caller, b->ev_out, 0) != hipSuccess)
    return fail(SFFT_EDEVICE);
  return SFFT_OK;
}

int32_t sfft_exec_batch_profile(const sfft_plan_t *plans, const void *const *xs,
                                int64_t *const *idx, void *const *vals, int64_t *d_counts,
                                int32_t *d_status, int32_t n, float *ms, int32_t *kernel,
                                int32_t cap) {
  // make sure the batch context exists and holds these pointers (no launch)
  int32_t rc = sfft_exec_batch_ex(plans, xs, idx, vals, d_counts, d_status, n, nullptr,
                                  SFFT_BATCH_NO_GRAPH | kBatchPrepareOnly);
  if (rc != SFFT_OK) return rc;
  std::lock_guard<std::mutex> lk(g_batch_mu);
  std::vector<const sfft_plan_s *> key(plans, plans + n);
  BatchCtx *b = g_batches[key].get();
  LaunchCtx c = b->lc;
  c.io = b->io_dev();
  Prof prof;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(SFFT_EDEVICE);
  const hipError_t le = b->launch_all(c, b->stream, &prof);
  const hipError_t se = hipStreamSynchronize(b->stream);
  int32_t cnt = 0;
  if (le == hipSuccess && se == hipSuccess) {
    for (size_t i = 1; i < prof.ev.size() && cnt < cap; i++, cnt++) {
      float t = 0.f;
      (void)hipEventElapsedTime(&t, prof.ev[i - 1], prof.ev[i]);
      if (ms) ms[cnt] = t;
      if (kernel) kernel[cnt] = prof.id[i];
    }
  }
  for (hipEvent_t e : prof.ev) (void)hipEventDestroy(e);
  if (le != hipSuccess || se != hipSuccess) return fail(SFFT_EDEVICE);
  return cnt;
}

int32_t sfft_exec_batch(const sfft_plan_t *plans, const void *const *xs, int64_t *const *idx,
                        void *const *vals, int64_t *d_counts, int32_t *d_status, int32_t n,
                        void *stream) {
  return sfft_exec_batch_ex(plans, xs, idx, vals, d_counts, d_status, n, stream, 0);
}

int32_t sfft_bucketize(sfft_plan_t plan, const void *x, void *out) {
  if (!plan) return fail(SFFT_EINVAL);
  if (!is_device_ptr(x) || !is_device_ptr(out)) return fail(SFFT_EINVAL);
  int32_t rc;
  BatchCtx *b = single_ctx(plan, &rc);
  if (!b) return fail(rc);
  LaunchCtx c = b->lc;
  c.io = nullptr;
  c.io1.x = (const float2 *)x;
  c.io1.count = b->count_dev();
  c.io1.status = b->status_dev();
  if (launch_reset(c, nullptr) != hipSuccess || launch_level0(c, nullptr) != hipSuccess ||
      launch_export_level0(c, out, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return fail(SFFT_EDEVICE);
  return SFFT_OK;
}

static void fill_stats(const SigState &st, const SigDesc &d, int64_t count, int32_t status,
                       sfft_stats_t *out) {
  out->count = count;
  out->status = status;
  out->levels = st.levels;
  out->samples = st.samples;
  out->found = st.found;
  out->noise_var = st.noise_var;
  out->sref2 = st.sref2;
  out->level_mask = st.level_mask;
  out->ident = d.kind == SFFT_KIND_FFAST ? st.ident : 0;
  out->h2d_bytes = 0;
}

int64_t sfft_exec_host(sfft_plan_t plan, const void *x, int64_t *out_idx, void *out_val,
                       sfft_stats_t *stats) {
  if (!plan || !x || !out_idx || !out_val) return fail(SFFT_EINVAL);
  if (is_device_ptr(x) || is_device_ptr(out_idx) || is_device_ptr(out_val)) return fail(SFFT_EINVAL);
  if (plan->info.sample_format != SFFT_SAMPLES_C64) return fail(SFFT_EUNSUPPORTED);
  int32_t rc;
  HostCtx *h = host_ctx(plan, &rc);
  if (!h) return fail(rc);
  BatchCtx &b = h->b;
  const int64_t K = plan->info.K;
  LaunchCtx c = b.lc;
  c.io = nullptr;
  c.io1.x = (const float2 *)h->img.p;
  c.io1.idx = (int64_t *)h->res.p;
  c.io1.val = (float2 *)((int64_t *)h->res.p + K);
  c.io1.count = b.count_dev();
  c.io1.status = b.status_dev();
  const hipStream_t s = h->stream;
  const float2 *xh = (const float2 *)x;
  int64_t moved = 0;
  auto stage = [&](int level) -> int32_t {
    const int64_t n = level_samples(plan, level);
    const int32_t r = h->reserve((size_t)n);
    if (r != SFFT_OK) return r;
    gather_samples(plan, level, xh, h->staging, n, h->pool.get());
    if (hipMemcpyAsync(h->packed.p, h->staging, sizeof(float2) * (size_t)n, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        launch_scatter(c.desc, level, (const float2 *)h->packed.p, n, (float2 *)h->img.p, s) != hipSuccess)
      return SFFT_EDEVICE;
    moved += n * (int64_t)sizeof(float2);
    return SFFT_OK;
  };
  if ((rc = stage(0)) != SFFT_OK) return fail(rc);
  if (launch_reset(c, s) != hipSuccess || launch_level0(c, s) != hipSuccess) return fail(SFFT_EDEVICE);
  for (size_t i = 0; i < b.lay.levels.size(); i++) {
    const int l = (int)i + 1;
    const LevelLaunch &L = b.lay.levels[i];
    // the level's samples are fetched only if the scheduler opened it
    if (launch_sched(c, l, s) != hipSuccess ||
        hipMemcpyAsync(h->word, &c.st[0].level_mask, sizeof(uint64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(SFFT_EDEVICE);
    if (!((*h->word >> l) & 1ull)) break;
    if ((rc = stage(l)) != SFFT_OK) return fail(rc);
    if ((L.fft && launch_expand_fft(c, l, L.grid_fft, s) != hipSuccess) ||
        (L.direct && launch_expand_direct(c, l, L.grid_direct, s) != hipSuccess) ||
        (L.children && launch_children(c, l, L.grid_children, s) != hipSuccess))
      return fail(SFFT_EDEVICE);
  }
  int64_t cnt = 0;
  int32_t status = 0;
  SigState st;
  if (launch_finalize(c, s) != hipSuccess ||
      hipMemcpyAsync(out_idx, c.io1.idx, sizeof(int64_t) * (size_t)K, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(out_val, c.io1.val, sizeof(float2) * (size_t)K, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&cnt, c.io1.count, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&status, c.io1.status, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&st, b.st_dev(), sizeof(SigState), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(SFFT_EDEVICE);
  if (stats) {
    fill_stats(st, b.lay.desc[0], cnt, status, stats);
    stats->h2d_bytes = moved;
  }
  return cnt;
}

int32_t sfft_exec_stats(sfft_plan_t plan, sfft_stats_t *out) {
  if (!plan || !out || !plan->single) return fail(SFFT_EINVAL);
  BatchCtx *b = plan->single.get();
  SigState st;
  int64_t cnt = 0;
  int32_t status = 0;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(&st, b->st_dev(), sizeof(SigState), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&cnt, b->count_dev(), sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&status, b->status_dev(), sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(SFFT_EDEVICE);
  fill_stats(st, b->lay.desc[0], cnt, status, out);
  return SFFT_OK;
}

int32_t sfft_batch_stats(const sfft_plan_t *plans, int32_t n, int32_t i, sfft_stats_t *out) {
  if (!plans || n < 1 || i < 0 || i >= n || !out) return fail(SFFT_EINVAL);
  std::lock_guard<std::mutex> lk(g_batch_mu);
  std::vector<const sfft_plan_s *> key(plans, plans + n);
  auto it = g_batches.find(key);
  if (it == g_batches.end()) return fail(SFFT_EINVAL);
  BatchCtx *b = it->second.get();
  SigState st;
  int64_t cnt = 0;
  int32_t status = 0;
  const SigIO &io = b->io_last[i];
  if (hipStreamSynchronize(b->stream) != hipSuccess ||
      hipMemcpy(&st, b->st_dev() + i, sizeof(SigState), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&cnt, io.count, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&status, io.status, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(SFFT_EDEVICE);
  fill_stats(st, b->lay.desc[i], cnt, status, out);
  return SFFT_OK;
}

int32_t sfft_workspace(const sfft_plan_t *plans, int32_t n, sfft_workspace_t *out,
                       sfft_workspace_signal_t *sig) {
  if (!plans || n < 1 || !out) return fail(SFFT_EINVAL);
  std::vector<const sfft_plan_s *> key(plans, plans + n);
  for (int i = 0; i < n; i++)
    if (!plans[i]) return fail(SFFT_EINVAL);
  Layout Y;
  const int32_t rc = make_layout(key, false, 256, Y);
  if (rc != SFFT_OK) return fail(rc);
  out->bytes = (int64_t)Y.bytes;
  out->y0 = Y.n_y0;
  out->fst = Y.n_fst;
  out->found = Y.n_found;
  out->multi = Y.n_multi;
  out->multi_vec = Y.n_mvec;
  out->jacc = Y.n_jacc;
  out->jcol = Y.n_jcol;
  out->nmax = Y.nmax;
  out->jstride = kJumpMax;
  out->levels = (int32_t)Y.levels.size();
  out->nsig = n;
  if (sig)
    for (int i = 0; i < n; i++) {
      const SigDesc &d = Y.desc[i];
      sfft_workspace_signal_t &w = sig[i];
      memset(&w, 0, sizeof(w));
      w.y0_off = d.y0_off;
      w.fst_off = d.fst_off;
      w.found_off = d.found_off;
      w.multi_off = d.multi_off;
      w.jcol_off = d.jc_off;
      w.found_cap = d.found_cap;
      w.multi_cap = d.multi_cap;
      w.col_rows = d.l1 ? d.col_rows : 0;
      w.n = d.n;
      w.l1 = d.l1;
      w.jump_L = d.jump_L;
    }
  return SFFT_OK;
}

void sfft_release_batches(void) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  g_batches.clear();
}

int32_t sfft_last_error(void) { return g_last_error; }

const char *sfft_strerror(int32_t code) {
  switch (code) {
    case SFFT_OK: return "ok";
    case SFFT_EINVAL: return "invalid argument";
    case SFFT_EUNSUPPORTED: return "unsupported size or factorisation";
    case SFFT_ENOMEM: return "device allocation failed";
    case SFFT_EDEVICE: return "HIP runtime or kernel launch error";
    case SFFT_ETOOBIG: return "workspace larger than the static scratch of sfft_exec_noalloc";
    default: return "unknown error";
  }
}

}  // extern "C"
