// C-ABI of libsbs: argument checks, workspace layout, plan choice, launch
// sequences and the autotuner. The operation is defined in include/sbs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/sbs.h"
#include "sbs_internal.h"

namespace sbs {
hipError_t launch_put_desc(FrameDev* table, const FrameDev* host, int nframes, hipStream_t s);
hipError_t launch_prologue(const FrameDev* table, int f0, int nf, int max_rows, WsHeader* hdr,
                           hipStream_t s);
hipError_t launch_finalize(const FrameDev* table, int f0, int nf, hipStream_t s);
hipError_t launch_tile_grid(const FrameDev* table, int fi, int64_t nitems, int chunk, bool wide, hipStream_t s);
hipError_t launch_tile_persistent(const FrameDev* table, int nframes, const QueueTotals& totals, int chunk, bool wide,
                                  int grid, WsHeader* hdr, hipStream_t s);
hipError_t launch_ref(const uint8_t* L, const uint8_t* R, int W, int H, int C, int64_t pitch, const uint32_t* idx,
                      int64_t n, int r, int dmax, uint8_t* od, uint32_t* oc, uint32_t* err, hipStream_t s);
}  // namespace sbs

namespace {
thread_local std::string g_err;
}  // namespace

namespace sbs {
int report_error(int status, const char* msg) {
  g_err = msg;
  return status;
}
}  // namespace sbs

using namespace sbs;

namespace {

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SBS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------- device info
struct DevInfo {
  bool checked = false;
  bool ok = false;
  int cus = 0;
  std::string arch;
};
std::mutex g_mu;
std::map<int, DevInfo> g_dev;

int device_check(int* cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  DevInfo& d = g_dev[dev];
  if (!d.checked) {
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    d.arch = p.gcnArchName;
    d.cus = p.multiProcessorCount;
    d.ok = d.arch.rfind("gfx950", 0) == 0;
    d.checked = true;
  }
  if (!d.ok) return fail(SBS_ERR_UNSUPPORTED, "device %d is %s, not gfx950", dev, d.arch.c_str());
  if (cus) *cus = d.cus;
  return SBS_OK;
}

// ---------------------------------------------------------------- plans
struct Plan {
  int cpl = 4, chunk = 8, ty = 64, wpc = 16;
};
bool g_forced = false;
Plan g_forced_plan;
std::map<std::string, Plan> g_tuned;

int density_bucket(const sbs_frame& f) {
  double rho = (double)f.n / ((double)f.W * f.H);
  int b = (int)(rho * 20.0);  // 5% buckets
  return b > 20 ? 20 : b;
}

// Frames per launch, rounded up to a power of two: a plan tuned for a
// 250-frame batch (few, large items per wavefront slot) is not the plan of a
// single frame of the same shape.
int batch_bucket(int nframes) {
  int b = 1;
  while (b < nframes && b < (1 << 20)) b <<= 1;
  return b;
}

std::string plan_key(const sbs_frame& f, int nframes) {
  std::ostringstream o;
  o << "gfx950/" << f.W << "x" << f.H << "x" << f.C << "/b" << f.block << "/d" << f.dmax << "/rho"
    << density_bucket(f) << "/nf" << batch_bucket(nframes);
  return o.str();
}

bool packs(const sbs_frame& f) { return 2 * (int64_t)f.block * 255 * f.C <= 65535; }

// The tile kernel packs a row's list range as (first - tile's first slot) <<
// shift | count, with shift 8 (4 columns per lane) or 9 (8 columns per
// lane); the offset is at most min(n, (tile rows - 1) x W).
bool ranges_fit(const sbs_frame& f, int ty, int shift) {
  return std::min<int64_t>(f.n, (int64_t)(ty - 1) * f.W) < (1LL << (32 - shift));
}

// Window columns per lane that frame f runs with under plan p: 8 needs
// 8-disparity chunks, packed accumulators and row list ranges that fit; 4
// otherwise.
int cpl_of(const sbs_frame& f, int plan_cpl, int chunk, int ty) {
  return plan_cpl == 8 && chunk == 8 && packs(f) && ranges_fit(f, ty, 9) ? 8 : 4;
}

// Tile rows of frame f under a plan of `ty` rows: halved until its row list
// ranges fit (only very wide frames with very long lists need that).
int ty_of(const sbs_frame& f, int ty, int cpl) {
  while (ty > 1 && !ranges_fit(f, ty, cpl == 8 ? 9 : 8)) ty /= 2;
  return ty;
}

// Work items of frame f with a given disparity chunk, tile height and lane width.
int64_t items_of(const sbs_frame& f, int chunk, int ty, int cpl = 4) {
  if (f.n <= 0) return 0;
  const int r = (f.block - 1) / 2;
  const int lpad = (r + 4) & ~3;
  const int c = cpl_of(f, cpl, chunk, ty);
  const int txo = (kWave * c - lpad - r) & ~3;
  const int t = ty_of(f, ty, c);
  return (int64_t)((f.W + txo - 1) / txo) * ((f.H + t - 1) / t) * ((f.dmax + chunk) / chunk);
}

// Default plan for the frames one launch covers: the largest items that
// still give the chip at least four work items per wavefront slot (256 CUs x
// 16), tried in the order (16 disparities, 128 rows), then 8 disparities with
// 128, 64 and 32 rows; 8 x 32 below that. Larger items amortise the window
// warm-up and the per-item work; more items balance the load (measured: one
// 4096x2304 frame runs 8% faster with 8 x 32 items than with 8 x 128, a
// 1390x1110 frame 44% faster; 250 such frames run best with 16 x 128).
Plan default_plan(const sbs_frame* frames, int nframes) {
  auto items = [&](int chunk, int ty) {
    int64_t t = 0;
    for (int i = 0; i < nframes; ++i) t += items_of(frames[i], chunk, ty, 4);
    return t;
  };
  const int64_t want = 4LL * 256 * 16;
  Plan p;
  p.wpc = 16;
  if (items(16, 128) >= want) { p.chunk = 16; p.ty = 128; return p; }
  p.chunk = 8;
  for (int ty : {128, 64, 32})
    if (items(8, ty) >= want) { p.ty = ty; return p; }
  p.ty = 32;
  return p;
}

// The plan of one launch over `frames` (keyed for the tuning cache by the
// first frame with work).
Plan choose_plan(const sbs_frame* frames, int nframes, const sbs_frame& key) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_forced) {
    Plan p = default_plan(frames, nframes);
    if (g_forced_plan.cpl) p.cpl = g_forced_plan.cpl;
    if (g_forced_plan.chunk) p.chunk = g_forced_plan.chunk;
    if (g_forced_plan.ty) p.ty = g_forced_plan.ty;
    if (g_forced_plan.wpc) p.wpc = g_forced_plan.wpc;
    return p;
  }
  auto it = g_tuned.find(plan_key(key, nframes));
  if (it != g_tuned.end()) return it->second;
  return default_plan(frames, nframes);
}

// ---------------------------------------------------------------- validation + layout
int validate(const sbs_frame& f, int i) {
  if (f.n < 0) return fail(SBS_ERR_INVALID_ARG, "frame %d: n < 0", i);
  if (f.n > INT32_MAX) return fail(SBS_ERR_INVALID_ARG, "frame %d: n > 2^31-1", i);
  if (f.W < 1 || f.H < 1) return fail(SBS_ERR_INVALID_ARG, "frame %d: W and H must be >= 1", i);
  if ((int64_t)f.W * f.H > INT32_MAX) return fail(SBS_ERR_INVALID_ARG, "frame %d: W*H >= 2^31", i);
  if (f.C != 1 && f.C != 3) return fail(SBS_ERR_INVALID_ARG, "frame %d: C must be 1 or 3", i);
  if (f.pitch_bytes < (int64_t)f.W * f.C) return fail(SBS_ERR_INVALID_ARG, "frame %d: pitch < W*C", i);
  if (f.block < 1 || (f.block % 2) == 0) return fail(SBS_ERR_INVALID_ARG, "frame %d: block must be odd and >= 1", i);
  if (f.dmax < 0 || f.dmax > 255) return fail(SBS_ERR_INVALID_ARG, "frame %d: dmax must be in [0, 255]", i);
  if (f.n > 0 && (!f.left || !f.right || !f.boundary_idx || !f.out_disp))
    return fail(SBS_ERR_INVALID_ARG, "frame %d: NULL pointer with n > 0", i);
  if (f.block > SBS_MAX_BLOCK) return fail(SBS_ERR_UNSUPPORTED, "frame %d: block %d > %d", i, f.block, SBS_MAX_BLOCK);
  return SBS_OK;
}

struct FrameLayout {
  size_t map_off, keys_off, lp_off, rp_off, rb_off, state_off, tptr_off, end;
  int lpw, rpw, ph, lpad, rpad, rbw, txo, ntx, tpw;
};

// Layout of one frame's part of the workspace for tiles of `span` window
// columns (64 x columns per lane); a tile's window columns start lpad > r
// columns left of its first output column.
FrameLayout frame_layout(const sbs_frame& f, size_t base, int span) {
  FrameLayout L;
  const int r = (f.block - 1) / 2;
  // Left copy: image column c at c + lpad; right copy: at c + rpad. Both pads
  // are multiples of 4 so 4-pixel groups stay 16-byte aligned; rpad leaves room
  // for the largest disparity chunk to the left of column 0. A tile reads
  // `span` columns from its first window column on.
  L.lpad = (r + 4) & ~3;
  L.rpad = (L.lpad + f.dmax + kMaxChunk + 1 + 3) & ~3;
  L.lpw = (int)align_up((size_t)f.W + span, 64);
  L.rpw = (int)align_up((size_t)f.W + span + L.rpad, 64);
  L.ph = f.H + 2 * r;
  const int groups = (f.W + 63) / 64;
  L.rbw = (groups + 63) / 64;
  size_t o = align_up(base, 256);
  L.map_off = o; o = align_up(o + (size_t)f.W * f.H * 4, 256);
  L.keys_off = o; o = align_up(o + (size_t)std::max<int64_t>(f.n, 1) * 4, 256);
  // One spare padded row at the bottom: the tile kernel's last prefetch reads it and discards it.
  L.lp_off = o; o = align_up(o + (size_t)L.lpw * (L.ph + 1) * 4, 256);
  L.rp_off = o; o = align_up(o + (size_t)L.rpw * (L.ph + 1) * 4, 256);
  L.rb_off = o; o = align_up(o + (size_t)f.H * L.rbw * 8, 256);
  L.txo = (span - L.lpad - r) & ~3;
  L.ntx = (f.W + L.txo - 1) / L.txo;
  L.tpw = L.ntx + 1;
  L.state_off = o; o = align_up(o + 16, 256);
  L.tptr_off = o; o = align_up(o + (size_t)f.H * L.tpw * 4, 256);
  L.end = o;
  return L;
}

size_t table_bytes(int nframes) { return align_up(sizeof(FrameDev) * (size_t)std::max(nframes, 1), 256); }

// Workspace bytes for frames laid out with `spans[i]` window columns per
// tile (NULL: the widest tiles, which bounds every plan).
size_t total_bytes(const sbs_frame* frames, int nframes, const int* spans = nullptr) {
  size_t o = kHeaderBytes + table_bytes(nframes);
  for (int i = 0; i < nframes; ++i) o = frame_layout(frames[i], o, spans ? spans[i] : kMaxSpan).end;
  return o;
}

// ---------------------------------------------------------------- library-managed workspace
struct OwnWs {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::map<int, OwnWs> g_ws;

int own_workspace(size_t need, void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  OwnWs& w = g_ws[dev];
  if (w.bytes < need) {
    if (w.ptr) {
      e = hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      hipFree(w.ptr);
      w.ptr = nullptr;
      w.bytes = 0;
    }
    size_t sz = std::max(need, (size_t)1 << 20);
    e = hipMalloc(&w.ptr, sz);
    if (e != hipSuccess) return fail(SBS_ERR_WORKSPACE, "hipMalloc(%zu): %s", sz, hipGetErrorString(e));
    e = hipMemset(w.ptr, 0, kHeaderBytes);
    if (e != hipSuccess) return hip_fail(e, "hipMemset");
    w.bytes = sz;
  }
  *out = w.ptr;
  return SBS_OK;
}

void* own_workspace_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find(dev);
  return it == g_ws.end() ? nullptr : it->second.ptr;
}

// ---------------------------------------------------------------- kernel timing
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;

void timing_begin(hipStream_t s, hipEvent_t* a) {
  *a = nullptr;
  if (!g_timing) return;
  if (hipEventCreate(a) != hipSuccess) { *a = nullptr; return; }
  hipEventRecord(*a, s);
}

void timing_end(hipStream_t s, hipEvent_t a) {
  if (!a) return;
  hipEvent_t b;
  if (hipEventCreate(&b) != hipSuccess) { hipEventDestroy(a); return; }
  hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(g_mu);
  g_events.emplace_back(a, b);
}

// ---------------------------------------------------------------- run
enum Mode { kSingle = 0, kBatched = 1, kPerFrame = 2 };

int run(const sbs_frame* frames, int nframes, void* workspace, size_t ws_bytes, hipStream_t s, Mode mode,
        bool timed = true) {
  if (nframes < 0 || (nframes > 0 && !frames)) return fail(SBS_ERR_INVALID_ARG, "bad frame array");
  for (int i = 0; i < nframes; ++i) {
    int st = validate(frames[i], i);
    if (st != SBS_OK) return st;
  }
  int64_t live = 0;
  for (int i = 0; i < nframes; ++i) live += frames[i].n;
  if (live == 0) return SBS_OK;
  // Test hook: SBS_TEST_FAIL=launch makes the call fail as a failed launch
  // would, after validation and before any device work.
  if (const char* tf = getenv("SBS_TEST_FAIL"))
    if (std::strcmp(tf, "launch") == 0) return fail(SBS_ERR_HIP, "injected launch failure (SBS_TEST_FAIL)");
  int cus = 0;
  int st = device_check(&cus);
  if (st != SBS_OK) return st;

  // One plan per call (from the first frame with work): the persistent kernel is one instance.
  int lead = 0;
  while (lead < nframes && frames[lead].n == 0) ++lead;
  // One launch covers all frames in the batched kernel, one frame otherwise.
  const Plan plan = mode == kBatched ? choose_plan(frames, nframes, frames[lead])
                                     : choose_plan(frames + lead, 1, frames[lead]);
  std::vector<int> cpl((size_t)nframes), span((size_t)nframes);
  for (int i = 0; i < nframes; ++i) {
    cpl[(size_t)i] = cpl_of(frames[i], plan.cpl, plan.chunk, plan.ty);
    span[(size_t)i] = kWave * cpl[(size_t)i];
  }
  const size_t need = total_bytes(frames, nframes, span.data());
  if (workspace) {
    if (ws_bytes < need)
      return fail(SBS_ERR_INVALID_ARG, "workspace of %zu bytes < %zu needed", ws_bytes, need);
  } else {
    if (ws_bytes != 0) return fail(SBS_ERR_INVALID_ARG, "workspace NULL with nonzero size");
    st = own_workspace(need, &workspace);
    if (st != SBS_OK) return st;
  }
  char* base = (char*)workspace;
  WsHeader* hdr = (WsHeader*)base;
  FrameDev* table = (FrameDev*)(base + kHeaderBytes);

  std::vector<FrameDev> host((size_t)nframes);
  size_t off = kHeaderBytes + table_bytes(nframes);
  int64_t items = 0;
  QueueTotals qt{};
  int max_rows = 1;
  for (int i = 0; i < nframes; ++i) {
    const sbs_frame& f = frames[i];
    FrameLayout L = frame_layout(f, off, span[(size_t)i]);
    off = L.end;
    FrameDev& d = host[(size_t)i];
    std::memset(&d, 0, sizeof d);
    d.left = f.left;
    d.right = f.right;
    d.idx = f.boundary_idx;
    d.out_disp = f.out_disp;
    d.out_cost = f.out_cost;
    d.map = (int32_t*)(base + L.map_off);
    d.keys = (uint32_t*)(base + L.keys_off);
    d.lp = (uint32_t*)(base + L.lp_off);
    d.rp = (uint32_t*)(base + L.rp_off);
    d.rowbits = (uint64_t*)(base + L.rb_off);
    d.state = (uint32_t*)(base + L.state_off);
    d.tptr = (int32_t*)(base + L.tptr_off);
    d.tpw = L.tpw;
    d.pitch = f.pitch_bytes;
    d.n = f.n;
    d.W = f.W; d.H = f.H; d.C = f.C;
    d.r = (f.block - 1) / 2;
    d.pack = packs(f) ? 1 : 0;
    d.cpl = cpl[(size_t)i];
    d.linpl = (f.C == 3 && ((uintptr_t)f.left & 3) == 0 && (f.pitch_bytes & 3) == 0) ? 1 : 0;
    d.dmax = f.dmax;
    d.lpw = L.lpw; d.rpw = L.rpw; d.ph = L.ph; d.lpad = L.lpad; d.rpad = L.rpad; d.rbw = L.rbw;
    d.txo = L.txo;
    d.ty = ty_of(f, plan.ty, cpl[(size_t)i]);
    d.ntx = L.ntx;
    d.nty = (f.H + d.ty - 1) / d.ty;
    d.chunk = plan.chunk;
    d.nch = (f.dmax + 1 + plan.chunk - 1) / plan.chunk;
    d.item_base = items;
    d.nitems = f.n > 0 ? (int64_t)d.ntx * d.nty * d.nch : 0;
    items += d.nitems;
    const int64_t ntiles = f.n > 0 ? (int64_t)d.ntx * d.nty : 0;
    for (int q = 0; q < kQueues; ++q) {
      d.xbase[q] = qt.t[q];
      const int64_t tq = ntiles > q ? (ntiles - q + kQueues - 1) / kQueues : 0;
      qt.t[q] += tq * d.nch;
    }
    max_rows = std::max(max_rows, L.ph);
  }
  hipError_t e = launch_put_desc(table, host.data(), nframes, s);
  if (e != hipSuccess) return hip_fail(e, "descriptor upload");
  if (mode == kPerFrame || mode == kSingle) {
    for (int i = 0; i < nframes; ++i) {
      if (frames[i].n == 0) continue;
      e = launch_prologue(table, i, 1, host[(size_t)i].ph, hdr, s);
      if (e != hipSuccess) return hip_fail(e, "prologue");
      hipEvent_t ev = nullptr;
      if (timed) timing_begin(s, &ev);
      e = launch_tile_grid(table, i, host[(size_t)i].nitems, plan.chunk, cpl[(size_t)i] == 8, s);
      timing_end(s, ev);
      if (e != hipSuccess) return hip_fail(e, "tile kernel");
      e = launch_finalize(table, i, 1, s);
      if (e != hipSuccess) return hip_fail(e, "finalize");
    }
  } else {
    e = launch_prologue(table, 0, nframes, max_rows, hdr, s);
    if (e != hipSuccess) return hip_fail(e, "prologue");
    const bool wide = std::find(cpl.begin(), cpl.end(), 8) != cpl.end();
    // wide launches hold at most 12 wavefronts per CU (3 per SIMD)
    int64_t grid = (int64_t)cus * (wide ? std::min(plan.wpc, 12) : plan.wpc);
    if (grid > items) grid = items;
    hipEvent_t ev = nullptr;
    if (timed) timing_begin(s, &ev);
    e = launch_tile_persistent(table, nframes, qt, plan.chunk, wide, (int)std::max<int64_t>(grid, 1), hdr, s);
    timing_end(s, ev);
    if (e != hipSuccess) return hip_fail(e, "persistent tile kernel");
    e = launch_finalize(table, 0, nframes, s);
    if (e != hipSuccess) return hip_fail(e, "finalize");
  }
  return SBS_OK;
}

// ---------------------------------------------------------------- tuning cache (JSON)
std::string plan_json(const Plan& p) {
  std::ostringstream o;
  o << "{\"cols_per_lane\": " << p.cpl << ", \"chunk\": " << p.chunk << ", \"tile_rows\": " << p.ty
    << ", \"waves_per_cu\": " << p.wpc << "}";
  return o.str();
}

bool parse_int_field(const std::string& s, const char* name, int* out) {
  std::string pat = std::string("\"") + name + "\"";
  size_t p = s.find(pat);
  if (p == std::string::npos) return false;
  p = s.find(':', p);
  if (p == std::string::npos) return false;
  *out = std::atoi(s.c_str() + p + 1);
  return true;
}

int load_cache(const char* path) {
  std::ifstream in(path);
  if (!in) return fail(SBS_ERR_INVALID_ARG, "cannot open %s", path);
  std::stringstream ss;
  ss << in.rdbuf();
  std::string s = ss.str();
  size_t p = 0;
  std::map<std::string, Plan> got;
  while ((p = s.find('"', p)) != std::string::npos) {
    size_t q = s.find('"', p + 1);
    if (q == std::string::npos) break;
    std::string key = s.substr(p + 1, q - p - 1);
    size_t ob = s.find('{', q), cb = s.find('}', q);
    if (ob == std::string::npos || cb == std::string::npos || key.rfind("gfx", 0) != 0) { p = q + 1; continue; }
    std::string body = s.substr(ob, cb - ob + 1);
    Plan pl;
    if (parse_int_field(body, "cols_per_lane", &pl.cpl) && parse_int_field(body, "chunk", &pl.chunk) &&
        parse_int_field(body, "tile_rows", &pl.ty) && parse_int_field(body, "waves_per_cu", &pl.wpc))
      got[key] = pl;
    p = cb + 1;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : got) g_tuned[kv.first] = kv.second;
  return SBS_OK;
}

int save_cache(const char* path) {
  std::map<std::string, Plan> all;
  {
    std::ifstream in(path);
    if (in) { in.close(); load_cache(path); }
    std::lock_guard<std::mutex> lk(g_mu);
    all = g_tuned;
  }
  std::ofstream out(path);
  if (!out) return fail(SBS_ERR_INVALID_ARG, "cannot write %s", path);
  out << "{\n";
  size_t i = 0;
  for (auto& kv : all) {
    out << "  \"" << kv.first << "\": " << plan_json(kv.second) << (++i < all.size() ? ",\n" : "\n");
  }
  out << "}\n";
  return SBS_OK;
}

bool plan_valid(const Plan& p) {
  return (p.cpl == 4 || (p.cpl == 8 && p.chunk == 8)) && (p.chunk == 8 || p.chunk == 16) && p.ty >= 8 &&
         p.ty <= kMaxTileRows && p.wpc >= 1 && p.wpc <= 16;
}

}  // namespace

namespace sbs {
// For the fixed-scratch entry point (sbs_noalloc.hip): checks, workspace
// bound and the single-frame run into a caller-given buffer, without kernel
// timing (which creates events).
int validate_frame(const sbs_frame& f) { return validate(f, 0); }
size_t workspace_bound(const sbs_frame& f) { return total_bytes(&f, 1); }
int run_single_into(const sbs_frame& f, void* workspace, size_t ws_bytes, hipStream_t s) {
  return run(&f, 1, workspace, ws_bytes, s, kSingle, false);
}
int fail_message(int status, const char* msg) { return fail(status, "%s", msg); }
}  // namespace sbs

extern "C" {

int sbs_abi_version(void) { return SBS_ABI_VERSION; }

const char* sbs_last_error(void) { return g_err.c_str(); }

size_t sbs_workspace_bytes(const sbs_frame* frames, int32_t nframes) {
  if (nframes < 0 || (nframes > 0 && !frames)) return 0;
  for (int i = 0; i < nframes; ++i)
    if (validate(frames[i], i) != SBS_OK) return 0;
  return total_bytes(frames, nframes);
}

int sbs_sad_disparity(const uint8_t* left, const uint8_t* right, int32_t W, int32_t H, int32_t C,
                      int64_t pitch_bytes, const uint32_t* boundary_idx, int64_t n, int32_t block, int32_t dmax,
                      uint8_t* out_disp, uint32_t* out_cost, void* workspace, size_t workspace_bytes,
                      void* stream) {
  sbs_frame f{left, right, W, H, C, pitch_bytes, boundary_idx, n, block, dmax, out_disp, out_cost};
  return run(&f, 1, workspace, workspace_bytes, (hipStream_t)stream, kSingle);
}

int sbs_sad_disparity_batched(const sbs_frame* frames, int32_t nframes, void* workspace, size_t workspace_bytes,
                              void* stream) {
  return run(frames, nframes, workspace, workspace_bytes, (hipStream_t)stream, kBatched);
}

int sbs_sad_disparity_per_frame(const sbs_frame* frames, int32_t nframes, void* workspace, size_t workspace_bytes,
                                void* stream) {
  return run(frames, nframes, workspace, workspace_bytes, (hipStream_t)stream, kPerFrame);
}

int sbs_check_indices(const sbs_frame* frames, int32_t nframes, void* workspace, void* stream) {
  (void)frames;
  (void)nframes;
  if (!workspace) workspace = own_workspace_ptr();
  if (!workspace) return SBS_OK;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  uint32_t err = 0;
  e = hipMemcpy(&err, workspace, sizeof err, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  const uint32_t zero = 0;
  e = hipMemcpy(workspace, &zero, sizeof zero, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  if (err) return fail(SBS_ERR_INDEX_RANGE, "an index >= W*H was seen");
  return SBS_OK;
}

int sbs_sad_disparity_ref(const uint8_t* left, const uint8_t* right, int32_t W, int32_t H, int32_t C,
                          int64_t pitch_bytes, const uint32_t* boundary_idx, int64_t n, int32_t block,
                          int32_t dmax, uint8_t* out_disp, uint32_t* out_cost, void* stream) {
  sbs_frame f{left, right, W, H, C, pitch_bytes, boundary_idx, n, block, dmax, out_disp, out_cost};
  int st = validate(f, 0);
  if (st != SBS_OK) return st;
  if (n == 0) return SBS_OK;
  st = device_check(nullptr);
  if (st != SBS_OK) return st;
  void* ws = nullptr;
  st = own_workspace(kHeaderBytes, &ws);
  if (st != SBS_OK) return st;
  hipError_t e = launch_ref(left, right, W, H, C, pitch_bytes, boundary_idx, n, (block - 1) / 2, dmax, out_disp,
                            out_cost, &((WsHeader*)ws)->error, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "reference kernel");
  return SBS_OK;
}

int sbs_kernel_timing(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_timing = enable != 0;
  return SBS_OK;
}

int32_t sbs_kernel_times(float* ms, int32_t cap) {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    ev.swap(g_events);
  }
  int32_t n = 0;
  for (auto& pr : ev) {
    float t = -1.0f;
    if (hipEventSynchronize(pr.second) == hipSuccess) hipEventElapsedTime(&t, pr.first, pr.second);
    if (ms && n < cap) ms[n] = t;
    ++n;
    hipEventDestroy(pr.first);
    hipEventDestroy(pr.second);
  }
  return n;
}

int sbs_set_plan(const sbs_plan* plan) {
  if (!plan || (!plan->cols_per_lane && !plan->chunk && !plan->tile_rows && !plan->waves_per_cu)) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_forced = false;
    return SBS_OK;
  }
  Plan merged;  // fields left at 0 take the defaults for validation
  merged.cpl = plan->cols_per_lane ? plan->cols_per_lane : 4;
  merged.chunk = plan->chunk ? plan->chunk : 8;
  merged.ty = plan->tile_rows ? plan->tile_rows : 64;
  merged.wpc = plan->waves_per_cu ? plan->waves_per_cu : 16;
  if (!plan_valid(merged)) return fail(SBS_ERR_INVALID_ARG, "invalid plan");
  std::lock_guard<std::mutex> lk(g_mu);
  g_forced = true;
  g_forced_plan.cpl = plan->cols_per_lane;
  g_forced_plan.chunk = plan->chunk;
  g_forced_plan.ty = plan->tile_rows;
  g_forced_plan.wpc = plan->waves_per_cu;
  return SBS_OK;
}

int sbs_get_plan(const sbs_frame* frame, sbs_plan* plan) {
  if (!frame || !plan) return fail(SBS_ERR_INVALID_ARG, "NULL argument");
  int st = validate(*frame, 0);
  if (st != SBS_OK) return st;
  Plan p = choose_plan(frame, 1, *frame);   // as a single-frame call would plan it
  plan->cols_per_lane = p.cpl;
  plan->chunk = p.chunk;
  plan->tile_rows = p.ty;
  plan->waves_per_cu = p.wpc;
  return SBS_OK;
}

int sbs_get_plan_batched(const sbs_frame* frames, int32_t nframes, sbs_plan* plan) {
  if (!frames || nframes < 1 || !plan) return fail(SBS_ERR_INVALID_ARG, "NULL argument or no frames");
  for (int i = 0; i < nframes; ++i) {
    int st = validate(frames[i], i);
    if (st != SBS_OK) return st;
  }
  int lead = 0;
  while (lead < nframes - 1 && frames[lead].n == 0) ++lead;
  Plan p = choose_plan(frames, nframes, frames[lead]);   // as a batched call would plan it
  plan->cols_per_lane = p.cpl;
  plan->chunk = p.chunk;
  plan->tile_rows = p.ty;
  plan->waves_per_cu = p.wpc;
  return SBS_OK;
}

int sbs_load_tuning(const char* cache_path) {
  if (!cache_path) return fail(SBS_ERR_INVALID_ARG, "NULL path");
  return load_cache(cache_path);
}

int sbs_tune(const sbs_frame* frames, int32_t nframes, const char* cache_path) {
  if (nframes < 1 || !frames) return fail(SBS_ERR_INVALID_ARG, "no frames");
  for (int i = 0; i < nframes; ++i) {
    int st = validate(frames[i], i);
    if (st != SBS_OK) return st;
  }
  int st = device_check(nullptr);
  if (st != SBS_OK) return st;
  int lead = 0;   // the key frame, as a batched call picks it
  while (lead < nframes - 1 && frames[lead].n == 0) ++lead;
  bool was_forced;
  Plan was_plan;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    was_forced = g_forced;
    was_plan = g_forced_plan;
  }
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  Plan best;
  float best_ms = 1e30f;
  const int shapes[][2] = {{4, 8}, {4, 16}, {8, 8}};   // (columns per lane, disparity chunk)
  const int rows[] = {32, 64, 128, 256};
  const int wpcs[] = {4, 8, 16};
  // one frame: timed on the single-frame path (its own launch sequence, the
  // grid tile kernel), which calls on one frame take; more: the batched one
  // (the grid tile kernel has no persistent grid, so one wavefront count)
  const Mode tmode = nframes == 1 ? kSingle : kBatched;
  const int nwpc = tmode == kSingle ? 1 : 3;
  for (const auto& sh : shapes)
    for (int ty : rows)
      for (int wi = 0; wi < nwpc; ++wi) {
        const int w = tmode == kSingle ? Plan().wpc : wpcs[wi];
        Plan p;
        p.cpl = sh[0]; p.chunk = sh[1]; p.ty = ty; p.wpc = w;
        {
          std::lock_guard<std::mutex> lk(g_mu);
          g_forced = true;
          g_forced_plan = p;
        }
        st = run(frames, nframes, nullptr, 0, nullptr, tmode);  // warm-up (and workspace growth)
        if (st != SBS_OK) goto done;
        hipEventRecord(a, nullptr);
        for (int rep = 0; rep < 3; ++rep) {
          st = run(frames, nframes, nullptr, 0, nullptr, tmode);
          if (st != SBS_OK) goto done;
        }
        hipEventRecord(b, nullptr);
        hipEventSynchronize(b);
        float ms = 0;
        hipEventElapsedTime(&ms, a, b);
        if (ms < best_ms) { best_ms = ms; best = p; }
      }
done:
  hipEventDestroy(a);
  hipEventDestroy(b);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_forced = was_forced;
    g_forced_plan = was_plan;
    if (st == SBS_OK) g_tuned[plan_key(frames[lead], nframes)] = best;
  }
  if (st != SBS_OK) return st;
  if (cache_path) return save_cache(cache_path);
  return SBS_OK;
}

}  // extern "C"
