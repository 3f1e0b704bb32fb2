// HIP kernels for boundary-pixel SAD-WTA on gfx950.
//
// The operation (arXiv 2001.07809, Sec. III "Disparity Measurement of Boundary
// Pixels"; winner-takes-all, Sec. II): for each listed pixel, the disparity d
// in [0, dmax] that minimises the w x w (x channels) sum of absolute
// differences between the left window at x and the right window at x - d on
// the same rows, with replicate padding and ties to the smaller d.
//
// Tiled path (per frame; every kernel also runs over a whole batch of frames):
//   k_check     clears the result keys, answers indices >= W*H, finds out
//               whether the list is in strictly increasing raster order
//               (a repeated index sends it down the pixel-map path), and for
//               each row and tile column the first list slot at or after the
//               tile's first pixel (read by the tile kernel on ordered lists).
//   k_prep      replicate-padded RGBx copy of the right image (one u32 per
//               pixel, so one v_sad_u8 covers all channels of a pixel), and of
//               the left image: whole, or only the edge bands that tiles
//               reaching past an image edge read (RGB images in 4-byte-aligned
//               rows, which the other tiles read in place). For an unordered
//               list it also clears the pixel->slot map and row bits.
//   k_scatter   unordered lists: map[p] = largest slot k with idx[k] == p, and
//               per row one bit per 64-column group that holds a listed pixel.
//   k_tile_*    the column-sum kernel. One wavefront owns a tile of output
//               columns x rows and a chunk of disparities. Each lane owns four
//               adjacent window columns. Walking down the tile's rows it keeps,
//               per (column, disparity), the window-column sum of absolute
//               differences, updated with two v_sad_u8 per (column, disparity,
//               row): the row entering and the row leaving the window. On a row
//               that holds listed pixels it forms prefix sums along the row
//               (in-lane, then a DPP scan across lanes) in LDS; each listed
//               pixel reads its window sum as a difference of two prefix
//               entries and folds (cost << 8 | d) into its key with an atomic
//               minimum (the chunks of one tile run as separate work items).
//   k_finalize  splits keys into (disparity, cost) for every list entry.
// Reference path: k_ref evaluates each pixel by brute force straight from the
// original images, sharing nothing with the tiled path.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sbs_internal.h"

namespace sbs {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ uint32_t load_px(const uint8_t* row, int x, int C) {
  if (C == 1) return (uint32_t)row[x];
  const uint8_t* p = row + (int64_t)x * 3;
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
}

// Global-memory views (the descriptor's pointers are generic; these let the
// compiler emit global_load instead of flat_load).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 g_uint4;
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const u32x3 g_uint3;
typedef __attribute__((address_space(1))) const int32_t g_int32;
typedef __attribute__((address_space(1))) const uint32_t g_uint32;
typedef __attribute__((address_space(1))) const uint64_t g_uint64;
typedef __attribute__((address_space(1))) uint32_t g_uint32_rw;
typedef __attribute__((address_space(1))) u32x4 g_uint4_rw;

// ---------------------------------------------------------------------------
// Descriptor upload: the descriptors travel inside the kernel argument, so a
// captured graph replays them without touching host memory. Each frame's
// state words are reset here, before any kernel reads them.
__global__ void k_put_desc(FrameDev* table, DescBatch b) {
  int i = threadIdx.x;
  if (i < b.count) {
    table[b.first + i] = b.f[i];
    *b.f[i].state = 0u;
    *(uint64_t*)(b.f[i].state + 2) = (uint64_t)b.f[i].n;
  }
}

__global__ void k_reset_head(WsHeader* h) {
  if (threadIdx.x < kQueues) h->q[threadIdx.x].head = 0ull;
}

// Keys cleared, out-of-range entries answered (and the first such slot
// recorded), order checked, and the (row, tile column) list ranges of
// ordered lists found in the same pass: tptr[j] for the cell j = y * tpw + t
// (key K_j = y W + min(t txo, W)) is the first slot whose index reaches K_j,
// so entry k writes k into the cells whose keys lie in (idx[k-1], idx[k]]
// and the last entry writes n into the cells after it. For a list that
// turns out unordered the cells hold whatever its entries wrote; they are
// not read then.
// Four list entries per thread and step: 16-byte loads and stores where the
// caller's arrays allow them (idx 16-byte aligned; keys live in the
// workspace), entry by entry otherwise.
constexpr int64_t kShortRange = 8;   // list-range cells one thread writes alone
__global__ __launch_bounds__(256) void k_check(const FrameDev* __restrict__ table, int f0, WsHeader* hdr) {
  const FrameDev& f = table[f0 + blockIdx.y];
  const int64_t N = (int64_t)f.W * f.H, n = f.n;
  const uint32_t* idx = f.idx;
  uint32_t* keys = f.keys;
  const bool vec = ((uintptr_t)idx & 15u) == 0;
  bool unsorted = false;
  // cells with key <= p: y tpw + floor(x / txo) + 1 for p = y W + x < N
  // (the quotients from fp64 reciprocals, then corrected by one step)
  const int64_t cells = (int64_t)f.H * f.tpw;
  const uint32_t W = (uint32_t)f.W, txo = (uint32_t)f.txo;
  const double rw = 1.0 / (double)W, rt = 1.0 / (double)txo;
  auto cells_upto = [&](uint32_t p) -> int64_t {
    if ((int64_t)p >= N) return cells;
    uint32_t y = (uint32_t)((double)p * rw);
    if ((uint64_t)y * W > p) --y;
    else if ((uint64_t)(y + 1) * W <= p) ++y;
    const uint32_t x = p - y * W;
    uint32_t t = (uint32_t)((double)x * rt);
    if (t * txo > x) --t;
    else if ((t + 1) * txo <= x) ++t;
    return (int64_t)y * f.tpw + t + 1;
  };
  if (n == 0 && blockIdx.x == 0)
    for (int64_t j = threadIdx.x; j < cells; j += blockDim.x) f.tptr[j] = 0;
  for (int64_t k = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x); k < n; k += 4 * (int64_t)gridDim.x * blockDim.x) {
    uint32_t p[4] = {0u, 0u, 0u, 0u};
    if (vec && k + 3 < n) {
      const u32x4 v = *(g_uint4*)(idx + k);
      p[0] = v.x; p[1] = v.y; p[2] = v.z; p[3] = v.w;
      *(g_uint4_rw*)(keys + k) = u32x4{0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k + j < n) { p[j] = idx[k + j]; keys[k + j] = 0xFFFFFFFFu; }
    }
    const uint32_t prev = k > 0 ? idx[k - 1] : 0u;
    if (k > 0 && prev >= p[0]) unsorted = true;
    // cell ranges: entry k + j gets the cells from cells_upto(its predecessor)
    // to cells_upto(its index); the last entry's range reaches the end with
    // value n. Short ranges are written by their thread; long ones (a gap of
    // many empty rows) by all active lanes of the wavefront together.
    int64_t rlo[5], rhi[5];
    int32_t rv[5];
    {
      int64_t below = k == 0 ? 0 : cells_upto(prev);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        rlo[j] = rhi[j] = 0;
        rv[j] = (int32_t)(k + j);
        if (k + j < n) {
          const int64_t up = cells_upto(p[j]);
          rlo[j] = below;
          rhi[j] = up;
          below = up;
        }
      }
      const bool last = k <= n - 1 && n - 1 <= k + 3;
      rlo[4] = last ? below : 0;
      rhi[4] = last ? cells : 0;
      rv[4] = (int32_t)n;
    }
#pragma unroll
    for (int j = 0; j < 5; ++j)
      if (rhi[j] - rlo[j] <= kShortRange)
        for (int64_t c = rlo[j]; c < rhi[j]; ++c) f.tptr[c] = rv[j];
    const uint64_t act = __builtin_amdgcn_ballot_w64(true);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
    const int nact = __builtin_popcountll(act);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      uint64_t m = __builtin_amdgcn_ballot_w64(rhi[j] - rlo[j] > kShortRange);
      while (m) {
        const int lead = __builtin_ctzll(m);
        const int64_t lo = __shfl(rlo[j], lead, 64), hi = __shfl(rhi[j], lead, 64);
        const int32_t v = __shfl(rv[j], lead, 64);
        for (int64_t c = lo + rank; c < hi; c += nact) f.tptr[c] = v;
        m &= m - 1;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (k + j >= n) break;
      if (j < 3 && k + j + 1 < n && p[j] >= p[j + 1]) unsorted = true;
      if ((int64_t)p[j] >= N) {
        f.out_disp[k + j] = 255;
        if (f.out_cost) f.out_cost[k + j] = 0xFFFFFFFFu;
        atomicOr(&hdr->error, 1u);
        atomicMin((unsigned long long*)(f.state + 2), (unsigned long long)(k + j));
      }
    }
  }
  if (__builtin_amdgcn_ballot_w64(unsorted) && (threadIdx.x & 63) == 0) atomicOr(f.state, kUnsorted);
}

// Padded copies (and, for unordered lists, map and row-bit clearing). One
// block per padded row (grid-stride); each thread writes groups of four
// padded pixels with one 16-byte store. Groups that lie inside the image with
// a 4-byte-aligned source row read 12 (RGB) or 4 (gray) bytes with aligned
// dword loads; border groups and unaligned rows read pixel by pixel with
// clamped coordinates.
__device__ __forceinline__ u32x4 pack_group(const uint8_t* row, int ic0, int W, int C, bool aligned) {
  u32x4 o;
  if (aligned && ic0 >= 0 && ic0 + 3 < W) {
    if (C == 3) {
      const u32x3 q = *(g_uint3*)(row + (int64_t)ic0 * 3);   // one 12-byte load
      const uint32_t a = q.x, b = q.y, c = q.z;
      o.x = a & 0xFFFFFFu;
      o.y = (a >> 24) | ((b & 0xFFFFu) << 8);
      o.z = (b >> 16) | ((c & 0xFFu) << 16);
      o.w = c >> 8;
    } else {
      const uint32_t a = *(g_uint32*)(row + ic0);
      o.x = a & 0xFFu; o.y = (a >> 8) & 0xFFu; o.z = (a >> 16) & 0xFFu; o.w = a >> 24;
    }
  } else {
    o.x = load_px(row, clampi(ic0 + 0, 0, W - 1), C);
    o.y = load_px(row, clampi(ic0 + 1, 0, W - 1), C);
    o.z = load_px(row, clampi(ic0 + 2, 0, W - 1), C);
    o.w = load_px(row, clampi(ic0 + 3, 0, W - 1), C);
  }
  return o;
}

constexpr int kPrepBatch = 5;   // right-copy groups per thread in flight (a 4096-pixel row: 1128 groups)
__global__ __launch_bounds__(256) void k_prep(const FrameDev* __restrict__ table, int f0) {
  const FrameDev& f = table[f0 + blockIdx.y];
  const int W = f.W, H = f.H, C = f.C, r = f.r;
  const bool unsorted = (*f.state & kUnsorted) != 0;
  // Left copy groups written: all of them, or, where the tile kernel reads
  // the left image in place inside it, only the groups that windows reaching
  // past an image edge read (padded words below lpad + span, and from
  // W + lpad - span - 2 on, span being the widest tile of the frame).
  const int lg = f.lpw >> 2, span = kWave * f.cpl;
  const int band0 = f.linpl ? min((f.lpad + span) >> 2, lg) : lg;
  const int band1 = f.linpl ? min(max(band0, (W + f.lpad - span - 2) >> 2), lg) : lg;
  const int nl = band0 + (lg - band1);
  for (int v = blockIdx.x; v < f.ph; v += gridDim.x) {
    const int y = clampi(v - r, 0, H - 1);
    const uint8_t* lrow = f.left + (int64_t)y * f.pitch;
    const uint8_t* rrow = f.right + (int64_t)y * f.pitch;
    const bool la = ((uintptr_t)lrow & 3) == 0, ra = ((uintptr_t)rrow & 3) == 0;
    g_uint4_rw* lo = (g_uint4_rw*)(f.lp + (int64_t)v * f.lpw);
    g_uint4_rw* ro = (g_uint4_rw*)(f.rp + (int64_t)v * f.rpw);
    for (int g = threadIdx.x; g < nl; g += blockDim.x) {
      const int gg = g < band0 ? g : g - band0 + band1;
      lo[gg] = pack_group(lrow, 4 * gg - f.lpad, W, C, la);
    }
    const int ng = f.rpw >> 2;
    if (C == 3 && ra) {
      // RGB rows on 4-byte boundaries: kPrepBatch groups per thread with all
      // their 12-byte loads in flight together (one round trip to memory
      // for several groups, not one per group), border groups pixel by pixel
      for (int g0 = 0; g0 < ng; g0 += kPrepBatch * (int)blockDim.x) {
        u32x3 q[kPrepBatch];
#pragma unroll
        for (int u = 0; u < kPrepBatch; ++u) {
          const int g = g0 + u * (int)blockDim.x + (int)threadIdx.x, ic0 = 4 * g - f.rpad;
          if (g < ng && ic0 >= 0 && ic0 + 3 < W) q[u] = *(g_uint3*)(rrow + (int64_t)ic0 * 3);
        }
#pragma unroll
        for (int u = 0; u < kPrepBatch; ++u) {
          const int g = g0 + u * (int)blockDim.x + (int)threadIdx.x, ic0 = 4 * g - f.rpad;
          if (g >= ng) break;
          if (ic0 >= 0 && ic0 + 3 < W) {
            u32x4 o;
            o.x = q[u].x & 0xFFFFFFu;
            o.y = (q[u].x >> 24) | ((q[u].y & 0xFFFFu) << 8);
            o.z = (q[u].y >> 16) | ((q[u].z & 0xFFu) << 16);
            o.w = q[u].z >> 8;
            ro[g] = o;
          } else {
            ro[g] = pack_group(rrow, ic0, W, C, ra);
          }
        }
      }
    } else {
      for (int g = threadIdx.x; g < ng; g += blockDim.x) ro[g] = pack_group(rrow, 4 * g - f.rpad, W, C, ra);
    }
    if (unsorted && v >= r && v < r + H) {
      int32_t* mrow = f.map + (int64_t)(v - r) * W;
      for (int u = threadIdx.x; u < W; u += blockDim.x) mrow[u] = -1;
      uint64_t* brow = f.rowbits + (int64_t)(v - r) * f.rbw;
      for (int u = threadIdx.x; u < f.rbw; u += blockDim.x) brow[u] = 0ull;
    }
  }
}

// Unordered lists: map[p] = max k with idx[k] == p; row bits set (one atomic
// OR per distinct word per wavefront).
__global__ __launch_bounds__(256) void k_scatter(const FrameDev* __restrict__ table, int f0) {
  const FrameDev& f = table[f0 + blockIdx.y];
  if (!(*f.state & kUnsorted)) return;
  const int64_t N = (int64_t)f.W * f.H;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
  for (int64_t kb = first; kb < f.n; kb += stride) {       // uniform per wavefront
    const int64_t k = kb + (threadIdx.x & 63);
    int64_t word = -1;
    uint64_t bit = 0;
    if (k < f.n) {
      const uint32_t p = f.idx[k];
      if ((int64_t)p < N) {
        atomicMax(&f.map[p], (int32_t)k);
        const int y = (int)(p / (uint32_t)f.W), x = (int)(p % (uint32_t)f.W);
        word = (int64_t)y * f.rbw + (x >> 12);
        bit = 1ull << ((x >> 6) & 63);
      }
    }
    bool pending = word >= 0;
    uint64_t pm;
    while ((pm = __builtin_amdgcn_ballot_w64(pending)) != 0) {
      const int leader = __builtin_ctzll(pm);
      const int64_t lw = __shfl(word, leader, 64);
      const bool mine = pending && word == lw;
      uint64_t acc = mine ? bit : 0ull;
      for (int off = 32; off >= 1; off >>= 1) acc |= __shfl_xor(acc, off, 64);
      if ((int)(threadIdx.x & 63) == leader) atomicOr((unsigned long long*)&f.rowbits[lw], (unsigned long long)acc);
      if (mine) pending = false;
    }
  }
}

// ---------------------------------------------------------------------------
// Wave-wide inclusive prefix sum with DPP: shifts within rows of 16 lanes,
// then broadcasts of lane 15 and lane 31 to the rows above.
#define SBS_DPP_STEP(v, ctrl, rmask) \
  (v) += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(v), (ctrl), (rmask), 0xf, false)

// Four independent scans with their steps interleaved, so each DPP read has
// other work between it and the write of its source.
__device__ __forceinline__ void wave_incl_scan4(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t& d) {
  SBS_DPP_STEP(a, 0x111, 0xf); SBS_DPP_STEP(b, 0x111, 0xf); SBS_DPP_STEP(c, 0x111, 0xf); SBS_DPP_STEP(d, 0x111, 0xf);
  SBS_DPP_STEP(a, 0x112, 0xf); SBS_DPP_STEP(b, 0x112, 0xf); SBS_DPP_STEP(c, 0x112, 0xf); SBS_DPP_STEP(d, 0x112, 0xf);
  SBS_DPP_STEP(a, 0x114, 0xf); SBS_DPP_STEP(b, 0x114, 0xf); SBS_DPP_STEP(c, 0x114, 0xf); SBS_DPP_STEP(d, 0x114, 0xf);
  SBS_DPP_STEP(a, 0x118, 0xf); SBS_DPP_STEP(b, 0x118, 0xf); SBS_DPP_STEP(c, 0x118, 0xf); SBS_DPP_STEP(d, 0x118, 0xf);
  SBS_DPP_STEP(a, 0x142, 0xa); SBS_DPP_STEP(b, 0x142, 0xa); SBS_DPP_STEP(c, 0x142, 0xa); SBS_DPP_STEP(d, 0x142, 0xa);
  SBS_DPP_STEP(a, 0x143, 0xc); SBS_DPP_STEP(b, 0x143, 0xc); SBS_DPP_STEP(c, 0x143, 0xc); SBS_DPP_STEP(d, 0x143, 0xc);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Keeps the row loop's steps in program order: an empty instruction that
// takes every accumulator as operand and clobbers memory, so neither the
// arithmetic on the accumulators nor loads and LDS traffic move across it.
template <int COLS, int N>
__device__ __forceinline__ void pin_step(uint32_t (&v)[COLS][N]) {
#pragma unroll
  for (int c = 0; c < COLS; ++c)
#pragma unroll
    for (int k = 0; k < N; k += 4)
      asm volatile("" : "+v"(v[c][k]), "+v"(v[c][k + 1]), "+v"(v[c][k + 2]), "+v"(v[c][k + 3])::"memory");
}

// Tile geometry of one lane width: COLS window columns per lane, a span of
// 64 * COLS window columns per wavefront, and G disparities whose prefix sums
// share the LDS at once (8 for 4 columns per lane, 4 for 8, so the LDS of one
// wavefront stays under 10 KB and 16 wavefronts fit a CU).
template <int COLS>
struct Geom {
  static constexpr int kSpanC = kWave * COLS;
  static constexpr int G = COLS == 8 ? 4 : 8;
  static constexpr int kTpShift = COLS == 8 ? 9 : 8;   // row ranges: count < 2^kTpShift
};

// LDS of one work item: prefix sums for G disparities and, for unordered
// lists (4 columns per lane only), the current row's listed pixels.
// pre[k][j] is the inclusive prefix sum over window columns 0..j. Windows
// never start at column 0 (the left margin lpad exceeds r), so no zero entry
// is needed, and a row is exactly 64 * COLS words: the same column of rows k
// and k + 1 lies a multiple of 256 bytes apart, which lets one ds_read2st64
// fetch both.
struct TileLds4 {
  uint32_t pre[8][kWave * 4] __attribute__((aligned(16)));
  union {
    struct {
      int16_t eo[kWave * 4];   // unordered lists: listed pixels of the row (output column offset)
      int32_t es[kWave * 4];   //                  and their representative slots
    };
    uint32_t tp[kMaxTileRows];   // ordered lists: list range of each row of the tile, packed
  };
};
struct TileLds8 {
  uint32_t pre[4][kWave * 8] __attribute__((aligned(16)));
  uint32_t tp[kMaxTileRows];
};
union TileLds {
  TileLds4 n;
  TileLds8 w;
};
static_assert(sizeof(TileLds) <= 9856, "LDS of one wavefront: 16 wavefronts per CU share 160 KB");
template <int COLS> struct LdsOf;
template <> struct LdsOf<4> { static __device__ __forceinline__ TileLds4& get(TileLds& s) { return s.n; } };
template <> struct LdsOf<8> { static __device__ __forceinline__ TileLds8& get(TileLds& s) { return s.w; } };

typedef __attribute__((address_space(3))) u32x4 lds_u32x4;

// The tile kernels run one wavefront per workgroup, and one wavefront's LDS
// operations complete in the order it issues them: a value one lane writes
// is seen by any later read of another lane. Ordering LDS traffic between
// phases of an item therefore needs only the compiler to keep the order (no
// wait for the writes to finish).
__device__ __forceinline__ void wave_lds_order() { asm volatile("" ::: "memory"); }

// The pixels one lane needs from one padded row: its COLS left columns, and
// the DC + COLS right columns that pair with them over the chunk (right
// index c + DC - k pairs with left column c at disparity d0 + k; index 0 is
// never used). Lane l's right words start at word COLS * l of the wave's
// span. Each lane loads all of them itself: neighbouring lanes read
// overlapping words, which the L1 cache serves, and that costs less than
// passing words between lanes with DPP shifts.
template <int DC, int COLS>
struct RowRegs {
  uint32_t L[COLS];
  uint32_t R[DC + COLS];
};

// Where a wave's left pixels come from. Copy: the padded RGBx copy, one
// 16-byte load per four columns. In place (tiles whose window lies inside the
// image, C = 3, 4-byte-aligned caller rows): the caller's RGB row, one 16-byte
// load at 12 bytes per four columns (its last 4 bytes belong to the next
// group), spread to RGBx words by v_perm_b32 once the load has arrived. The
// byte selectors are uniform; for the copy they leave the words as they are,
// so both sources take the same instructions.
struct LeftSrc {
  const char* base;   // row q of the source: base + clamp(q - roff, 0, qmax) * pitch
  int64_t pitch;
  int roff, qmax;
  uint32_t lb, gs;    // this lane's first byte in a row; bytes between its groups of four columns
  uint32_t s0, s1, s2, s3;   // v_perm_b32 selectors of the four words of a group
  __device__ __forceinline__ const char* row(int q) const {
    const int v = q - roff;
    return base + (int64_t)(v < 0 ? 0 : (v > qmax ? qmax : v)) * pitch;
  }
};

// A pointer that is the same in every lane, as a scalar value (in the
// out-of-line item functions the compiler cannot tell by itself).
__device__ __forceinline__ const char* wave_uniform(const void* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const char*)(((uint64_t)hi << 32) | lo);
}

// lrow, rrow: the wave's row bases (uniform), taken as scalars, so each load
// is the scalar base plus this lane's 32-bit byte offset (ls.lb on the left;
// rb = 4 * COLS * lane on the right) with no per-lane address arithmetic.
template <int DC, int COLS>
__device__ __forceinline__ void load_row(const char* lrow_, const LeftSrc& ls, const uint32_t* rrow, uint32_t rb,
                                         RowRegs<DC, COLS>& o) {
  const char* lrow = wave_uniform(lrow_);
  const char* rr = wave_uniform(rrow);
  // the offsets as opaque 32-bit values here, so each load is formed as
  // (scalar base, 32-bit lane offset) rather than from a 64-bit lane address
  uint32_t lb = ls.lb;
  asm volatile("" : "+v"(lb));
  asm volatile("" : "+v"(rb));
#pragma unroll
  for (int b = 0; b < COLS / 4; ++b) {
    const u32x4 lv = *(g_uint4*)(lrow + (lb + (uint32_t)b * ls.gs));
    o.L[4 * b] = lv.x; o.L[4 * b + 1] = lv.y; o.L[4 * b + 2] = lv.z; o.L[4 * b + 3] = lv.w;
  }
#pragma unroll
  for (int b = 0; b < (DC + COLS) / 4; ++b) {
    const u32x4 t = *(g_uint4*)(rr + rb + 16 * b);
    o.R[4 * b] = t.x; o.R[4 * b + 1] = t.y; o.R[4 * b + 2] = t.z; o.R[4 * b + 3] = t.w;
  }
}

// Left words of a loaded row to RGBx: word k of a group takes bytes of words
// k and k - 1 (word 0 only its own), highest word first, so each reads words
// not yet rewritten.
template <int DC, int COLS>
__device__ __forceinline__ void left_words(RowRegs<DC, COLS>& o, const LeftSrc& ls) {
#pragma unroll
  for (int b = 0; b < COLS / 4; ++b) {
    uint32_t* w = o.L + 4 * b;
    w[3] = __builtin_amdgcn_perm(w[3], w[2], ls.s3);
    w[2] = __builtin_amdgcn_perm(w[2], w[1], ls.s2);
    w[1] = __builtin_amdgcn_perm(w[1], w[0], ls.s1);
    w[0] = __builtin_amdgcn_perm(w[0], w[0], ls.s0);
  }
}

// Word 0 of the right columns is loaded (whole aligned blocks) but never used
// in the sums; it is kept live up to the row's use so that every load writes
// only live registers (a dead load destination that the compiler reused for
// other work would make it wait for that load, and with it for every load
// issued before it).
template <int DC, int COLS>
__device__ __forceinline__ void keep_word0(const RowRegs<DC, COLS>& o) {
  asm volatile("" ::"v"(o.R[0]));
}

// Accumulators per lane: kPack == false keeps one 32-bit sum per (column,
// disparity); kPack == true keeps disparities d0 + 2j and d0 + 2j + 1 of a
// column in the low and high 16 bits of one register (usable while the sum of
// two window columns, at most 2 * block * 255 * C, fits in 16 bits).
template <int DC, bool kPack, int COLS>
struct Acc {
  static constexpr int N = kPack ? DC / 2 : DC;
  uint32_t v[COLS][N];
  // window column COLS * lane + c, disparity d0 + k
  __device__ __forceinline__ uint32_t get(int c, int k) const {
    if constexpr (kPack) return (k & 1) ? (v[c][k >> 1] >> 16) : (v[c][k >> 1] & 0xFFFFu);
    else return v[c][k];
  }
  // sums over the lane's columns of disparities d0 + k and d0 + k + 1 (k even)
  __device__ __forceinline__ void total2(int k, uint32_t& t0, uint32_t& t1) const {
    if constexpr (kPack) {
      // column pairs added as 16-bit halves (no carry out of a half), then widened
      t0 = 0u;
      t1 = 0u;
#pragma unroll
      for (int p = 0; p < COLS / 2; ++p) {
        const u16x2 a = __builtin_bit_cast(u16x2, v[2 * p][k >> 1]) + __builtin_bit_cast(u16x2, v[2 * p + 1][k >> 1]);
        t0 += (uint32_t)a.x;
        t1 += (uint32_t)a.y;
      }
    } else {
      t0 = 0u;
      t1 = 0u;
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
        t0 += v[c][k];
        t1 += v[c][k + 1];
      }
    }
  }
};

// Adds one padded row to the accumulators.
template <int DC, bool kPack, int COLS>
__device__ __forceinline__ void add_row(RowRegs<DC, COLS>& a, Acc<DC, kPack, COLS>& acc, const LeftSrc& ls) {
  keep_word0(a);
  left_words(a, ls);
#pragma unroll
  for (int c = 0; c < COLS; ++c)
#pragma unroll
    for (int j = 0; j < Acc<DC, kPack, COLS>::N; ++j) {
      if constexpr (kPack)
        acc.v[c][j] = __builtin_amdgcn_sad_hi_u8(a.L[c], a.R[c + DC - 2 * j - 1],
                                                 __builtin_amdgcn_sad_u8(a.L[c], a.R[c + DC - 2 * j], acc.v[c][j]));
      else
        acc.v[c][j] = __builtin_amdgcn_sad_u8(a.L[c], a.R[c + DC - j], acc.v[c][j]);
    }
}

// Moves the window down one row: padded row `ex` leaves, `en` enters. The
// leaving row is taken off first, so no partial sum exceeds a full window.
template <int DC, bool kPack, int COLS>
__device__ __forceinline__ void slide_row(RowRegs<DC, COLS>& en, RowRegs<DC, COLS>& ex, Acc<DC, kPack, COLS>& acc,
                                          const LeftSrc& ls) {
  keep_word0(en);
  keep_word0(ex);
  left_words(ex, ls);
  left_words(en, ls);
#pragma unroll
  for (int c = 0; c < COLS; ++c)
#pragma unroll
    for (int j = 0; j < Acc<DC, kPack, COLS>::N; ++j) {
      if constexpr (kPack) {
        const uint32_t out = __builtin_amdgcn_sad_hi_u8(ex.L[c], ex.R[c + DC - 2 * j - 1],
                                                        __builtin_amdgcn_sad_u8(ex.L[c], ex.R[c + DC - 2 * j], 0u));
        const uint32_t t = acc.v[c][j] - out;   // no borrow between the halves: each half holds its own row
        acc.v[c][j] = __builtin_amdgcn_sad_hi_u8(en.L[c], en.R[c + DC - 2 * j - 1],
                                                 __builtin_amdgcn_sad_u8(en.L[c], en.R[c + DC - 2 * j], t));
      } else {
        const uint32_t out = __builtin_amdgcn_sad_u8(ex.L[c], ex.R[c + DC - j], 0u);
        acc.v[c][j] = __builtin_amdgcn_sad_u8(en.L[c], en.R[c + DC - j], acc.v[c][j] - out);
      }
    }
}

// One pass over output columns [xs, xe) of tile `tile` (row-major over the
// frame's ntx x nty tiles) for disparity chunk `chunk` (disparities
// chunk*DC .. +DC-1), COLS window columns per lane. Ordered lists take the
// whole tile in one pass; unordered lists may take a tile in several
// narrower passes. The window columns of the pass start lpad > r columns
// left of xs.
template <int DC, bool kSorted, bool kPack, int COLS>
__device__ __forceinline__ void tile_item_impl(const FrameDev& f, int tile, int chunk, int xs, int xe, TileLds& smu) {
  static_assert(COLS == 4 || (kSorted && kPack), "8 columns per lane: ordered lists, packed accumulators");
  constexpr int kSpanC = Geom<COLS>::kSpanC;
  constexpr int G = Geom<COLS>::G;
  constexpr int kTpShift = Geom<COLS>::kTpShift;
  constexpr int NB = kSorted ? COLS / 4 : 1;   // list entries of a row held in registers: 64 * NB
  auto& sm = LdsOf<COLS>::get(smu);
  // The lane index as an opaque value of this item: nothing derived from it
  // is hoisted out of the persistent kernel's item loop (where it would stay
  // live, in registers or spilled, across all items).
  int lane = threadIdx.x;
  asm volatile("" : "+v"(lane));
  // The descriptor's fields as values of this item: the row loop's compiler
  // barriers (pin_step) clobber memory, and fields read through `f` after
  // them would be loaded again.
  const uint32_t* const f_idx = f.idx;
  uint32_t* const f_keys = f.keys;
  // list entry k and key slot k: a scalar base plus an unsigned 32-bit byte
  // offset (k < 2^30), which keeps the pointers in scalar registers
  auto idx_at = [&](int k) -> uint32_t {
    return *(g_uint32*)((const char*)f_idx + (uint32_t)k * 4u);
  };
  const int32_t* const f_map = f.map;
  const int32_t* const f_tptr = f.tptr;
  const uint64_t* const f_rowbits = f.rowbits;
  const int f_tpw = f.tpw, f_rbw = f.rbw, f_ty = f.ty;
  const int tx = tile % f.ntx, tyi = tile / f.ntx;
  const int W = f.W, H = f.H, r = f.r;
  const int x0 = xs, y0 = tyi * f_ty;
  const int x1 = xe, y1 = min(y0 + f_ty, H);
  const int d0 = chunk * DC;
  const int dcount = min(DC, f.dmax + 1 - d0);
  const int lpad = f.lpad;
  constexpr bool sorted = kSorted;

  // Rows of this tile (up to kMaxTileRows = 256, four 64-bit masks) holding
  // a listed pixel in [x0, x1). Ordered lists: row y0 + 64 m + l's list range
  // goes to LDS (tp[64 m + l]), packed as (first - tbase) << kTpShift | count,
  // tbase being the first list slot of the tile's first row (count <= txo;
  // first - tbase <= min(n, (ty - 1) * W), which the host keeps below
  // 2^(32 - kTpShift)).
  const int tbase = kSorted ? f_tptr[(int64_t)y0 * f_tpw + tx] : 0;
  auto row_active = [&](int y, int& t0, int& t1) -> bool {
    if (y >= y1) return false;
    if (sorted) {
      const g_int32* tp = (g_int32*)(f_tptr + (int64_t)y * f_tpw + tx);
      t0 = tp[0];
      t1 = tp[1];
      return t1 > t0;
    }
    const int g0 = x0 >> 6, g1 = (x1 - 1) >> 6;
    bool a = false;
    for (int w = g0 >> 6; w <= (g1 >> 6); ++w) {
      const uint64_t bits = *(g_uint64*)(f_rowbits + (int64_t)y * f_rbw + w);
      const int lo = max(g0 - 64 * w, 0), hi = min(g1 - 64 * w, 63);
      const uint64_t m = (hi == 63 ? ~0ull : ((1ull << (hi + 1)) - 1)) & ~((1ull << lo) - 1);
      if (bits & m) a = true;
    }
    return a;
  };
  uint64_t rows[kMaxTileRows / 64];
#pragma unroll
  for (int m = 0; m < kMaxTileRows / 64; ++m) {
    int t0 = 0, t1 = 0;
    const bool act = (int)lane + 64 * m < f_ty && row_active(y0 + 64 * m + (int)lane, t0, t1);
    if constexpr (kSorted) sm.tp[64 * m + lane] = (uint32_t)(t0 - tbase) << kTpShift | (uint32_t)(t1 - t0);
    rows[m] = __builtin_amdgcn_ballot_w64(act);
  }
  // list range [first, first + count) of row y (uniform), from LDS
  auto row_range = [&](int y, int& first, int& count) {
    const uint32_t v = __builtin_amdgcn_readfirstlane(sm.tp[y - y0]);
    first = tbase + (int)(v >> kTpShift);
    count = (int)(v & ((1u << kTpShift) - 1u));
  };
  int ya = -1, yb = -1;
#pragma unroll
  for (int m = 0; m < kMaxTileRows / 64; ++m)
    if (ya < 0 && rows[m]) ya = y0 + 64 * m + __builtin_ctzll(rows[m]);
#pragma unroll
  for (int m = kMaxTileRows / 64 - 1; m >= 0; --m)
    if (yb < 0 && rows[m]) yb = y0 + 64 * m + 63 - __builtin_clzll(rows[m]);
  if (ya < 0) return;
  // first active row after y, or -1 (the masks are only indexed by constants,
  // so they stay in scalar registers)
  auto next_active = [&](int y) -> int {
    const int i = y - y0 + 1;
#pragma unroll
    for (int m = 0; m < kMaxTileRows / 64; ++m) {
      if (i >= 64 * (m + 1)) continue;
      const int sh = i > 64 * m ? i - 64 * m : 0;
      const uint64_t w = rows[m] >> sh;
      if (w) return y0 + 64 * m + sh + __builtin_ctzll(w);
    }
    return -1;
  };

  // Row bases (the same for the whole wave): padded row q of the pass (image
  // row q - r, clamped) starts at rp0 + q * rpw in the right copy, and at
  // ls.row(q) on the left (window column j is image column x0 - lpad + j);
  // lane l's right words start at byte lo = 4 * COLS * l. The left source is the
  // caller's image where the window lies inside it (with 2 columns to spare
  // for the last lane's 16-byte load), else the padded copy, which the
  // preparation writes for those windows.
  const uint32_t* rp0 = f.rp + x0 - lpad - d0 - DC + f.rpad;
  const uint32_t lo = 4u * COLS * (uint32_t)lane;   // byte offset of this lane's right words
  const int64_t rpw = f.rpw;
  LeftSrc ls;
  {
    const bool inpl = f.linpl && x0 >= lpad && x0 - lpad + Geom<COLS>::kSpanC + 2 <= W;
    ls.base = inpl ? (const char*)f.left + (int64_t)(x0 - lpad) * 3 : (const char*)(f.lp + x0);
    ls.pitch = inpl ? f.pitch : (int64_t)f.lpw * 4;
    ls.roff = inpl ? r : 0;
    ls.qmax = inpl ? H - 1 : f.ph;
    ls.gs = inpl ? 12u : 16u;
    ls.lb = ls.gs * (COLS / 4) * (uint32_t)lane;
    ls.s0 = inpl ? 0x0c020100u : 0x03020100u;
    ls.s1 = inpl ? 0x0c050403u : 0x07060504u;
    ls.s2 = inpl ? 0x0c040302u : 0x07060504u;
    ls.s3 = inpl ? 0x0c030201u : 0x07060504u;
  }

  // Disparities beyond dmax (last chunk only) never win: their keys are forced to ~0.
  uint32_t kill[DC];
#pragma unroll
  for (int k = 0; k < DC; ++k) kill[k] = k < dcount ? 0u : 0xFFFFFFFFu;

  // acc: per window column COLS * lane + c and disparity d0 + k, the sum over
  // the window's rows of the absolute differences (summed over channels).
  Acc<DC, kPack, COLS> acc;
#pragma unroll
  for (int c = 0; c < COLS; ++c)
#pragma unroll
    for (int j = 0; j < Acc<DC, kPack, COLS>::N; ++j) acc.v[c][j] = 0;

  int e0 = 0, cnt = 0;
  uint32_t pf_next[NB];                    // ordered lists: first 64 * NB list entries of the next active row
  int ob[NB];                              //                their output offsets, once the row is taken
  uint32_t idx2 = 0u;                      // ordered lists: list entry 64 * NB + lane of the row being taken
#pragma unroll
  for (int b = 0; b < NB; ++b) { pf_next[b] = 0u; ob[b] = 0; }
  int32_t mv[COLS];                        // unordered lists: pixel map of the next active row
  const uint32_t mlo = COLS * (uint32_t)lane;   // this lane's first window column
  // Deferred key update of the previous active row: lane l + 64 b < pend_cnt
  // holds the best of entry pend_e0 + l + 64 b in pend_best[b] (ordered
  // lists), or of slot pend_slot (unordered lists).
  uint32_t pend_best[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) pend_best[b] = 0xFFFFFFFFu;
  uint32_t pend_best2 = 0xFFFFFFFFu;       // ordered lists: entry 64 * NB + lane of the previous active row
  int pend_e0 = 0, pend_cnt = 0;
  int32_t pend_slot = -1;
  auto load_next = [&](int y) {            // list data of active row y (y < 0: none)
    if (y < 0) return;
    if constexpr (kSorted) {
      int t0, n0;
      row_range(y, t0, n0);
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if ((int)lane + 64 * b < n0) pf_next[b] = idx_at(t0 + (int)lane + 64 * b);
    } else {
      const int32_t* mrow = f_map + (int64_t)y * W + x0 - lpad;   // window column j -> image column x0 - lpad + j
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
        const int o = (int)mlo + c - lpad;
        mv[c] = (o >= 0 && x0 + o < x1) ? *(g_int32*)(mrow + mlo + c) : -1;
      }
    }
  };
  load_next(ya);   // in flight during the warm-up

  // Window of output row ya: padded rows ya .. ya + 2r (an odd count), in
  // pairs with the next row's loads in flight, then the last row.
  {
    const int last = ya + 2 * r;
    RowRegs<DC, COLS> A, B;
    load_row<DC, COLS>(ls.row(ya), ls, rp0 + ya * rpw, lo, A);
    for (int q = ya; q < last; q += 2) {
      load_row<DC, COLS>(ls.row(q + 1), ls, rp0 + (q + 1) * rpw, lo, B);
      add_row<DC, kPack, COLS>(A, acc, ls);
      load_row<DC, COLS>(ls.row(q + 2), ls, rp0 + (q + 2) * rpw, lo, A);
      add_row<DC, kPack, COLS>(B, acc, ls);
    }
    add_row<DC, kPack, COLS>(A, acc, ls);
  }

  // Row step y (y > ya first moves the window down from y - 1):
  //   slide          the vertical update: the one point where the wave waits
  //                  for memory, for the loads issued one step earlier;
  //   key update     of the previous active row, deferred to here so that it
  //                  is a full step old at the next wait;
  //   take_row(y)    the row's listed pixels from what that wait delivered,
  //                  then the loads for the next step and the next active row;
  //   per group of G disparities: prefix sums of the window to LDS, then the
  //                  window sums of the row's listed pixels as differences of
  //                  two prefix entries, folded into a running best.
  // Loaded values are only used after the wait of the slide, and the only
  // memory operations issued after the loads are rare (rows with more than
  // 64 * NB listed pixels in the tile).
  // prefix sums of disparities d0 + g .. d0 + g + G - 1 to LDS
  auto prefix_group = [&](int g) {
#pragma unroll
    for (int k0 = 0; k0 < G; k0 += 4) {
      // t: the lane's column total, then (after the wave scan) the prefix at
      // its last column; the columns before follow by subtraction, so no
      // in-lane prefixes stay live across the scan.
      uint32_t t[4];
      acc.total2(g + k0, t[0], t[1]);
      acc.total2(g + k0 + 2, t[2], t[3]);
      wave_incl_scan4(t[0], t[1], t[2], t[3]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        uint32_t o[COLS];
        o[COLS - 1] = t[i];
#pragma unroll
        for (int c = COLS - 1; c > 0; --c) o[c - 1] = o[c] - acc.get(c, g + k0 + i);
#pragma unroll
        for (int b = 0; b < COLS / 4; ++b) {
          u32x4 w;
          w.x = o[4 * b]; w.y = o[4 * b + 1]; w.z = o[4 * b + 2]; w.w = o[4 * b + 3];
          *(lds_u32x4*)&sm.pre[k0 + i][COLS * lane + 4 * b] = w;
        }
      }
    }
    wave_lds_order();
  };
  auto take_row = [&](int y) {
    cnt = 0;
    if constexpr (kSorted) {
      row_range(y, e0, cnt);
      // Turned into offsets here, before load_next reuses pf_next: the load of
      // the next row then writes the register this value occupied, and no
      // copy of a value still in flight (which would wait for every
      // outstanding load) is needed at the end of the step.
      const uint32_t rowbase = (uint32_t)y * (uint32_t)W + (uint32_t)x0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        ob[b] = (int)(pf_next[b] - rowbase);
        asm volatile("" : "+v"(ob[b])::"memory");
      }
      // The next 64 entries of a dense row, loaded before the step's row
      // loads: waiting for this load then leaves those in flight.
      if ((int)lane + kWave * NB < cnt) idx2 = idx_at(e0 + (int)lane + kWave * NB);
    } else {
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
        const uint64_t b = __builtin_amdgcn_ballot_w64(mv[c] >= 0);
        if (mv[c] >= 0) {
          const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
          sm.eo[pos] = (int16_t)(COLS * lane + c - lpad);
          sm.es[pos] = mv[c];
        }
        cnt += __builtin_popcountll(b);
      }
    }
  };
  // Best (cost << 8 | d) over group g of the listed pixel at output offset o
  // (0 <= o < x1 - x0; window columns o + lpad - r .. o + lpad + r).
  auto group_best = [&](int g, int o, uint32_t best) -> uint32_t {
    const int ih = o + lpad + r, il = o + lpad - r - 1;   // il >= 0: lpad > r
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const uint32_t s = sm.pre[k][ih] - sm.pre[k][il];
      best = min(best, ((s << 8) | (uint32_t)(d0 + g + k)) | kill[g + k]);
    }
    return best;
  };
  // a global (not flat) atomic: it counts only against the vector-memory counter
  auto key_min = [&](int32_t slot, uint32_t v) {
    __hip_atomic_fetch_min((g_uint32_rw*)((char*)f_keys + (uint32_t)slot * 4u), v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  };
  auto flush = [&]() {
    if constexpr (kSorted) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if ((int)lane + 64 * b < pend_cnt) key_min(pend_e0 + (int)lane + 64 * b, pend_best[b]);
      if ((int)lane + 64 * NB < pend_cnt) key_min(pend_e0 + (int)lane + 64 * NB, pend_best2);
      pend_cnt = 0;
    } else {
      if (pend_slot >= 0) key_min(pend_slot, pend_best[0]);
      pend_slot = -1;
    }
  };
  auto entries_row = [&](int y) {
    const uint32_t rowbase = (uint32_t)y * (uint32_t)W + (uint32_t)x0;
    bool has[NB];
    int32_t slot0 = -1;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      has[b] = (int)lane + 64 * b < cnt;
      if constexpr (!kSorted)
        if (has[b]) { ob[b] = sm.eo[lane]; slot0 = sm.es[lane]; }
    }
    uint32_t best[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) best[b] = 0xFFFFFFFFu;
    // Ordered lists: the next 64 entries of a dense row (entry 64 * NB + lane,
    // loaded when the row was taken) keep their best over the groups, with
    // one key update at the end; entries past those take one per group.
    constexpr int kHeld = kSorted ? NB + 1 : NB;
    const bool has2 = kSorted && (int)lane + kWave * NB < cnt;
    int o2 = 0;
    uint32_t best2 = 0xFFFFFFFFu;
    if (has2) o2 = (int)(idx2 - rowbase);
#pragma unroll
    for (int g = 0; g < DC; g += G) {
      prefix_group(g);
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (has[b]) best[b] = group_best(g, ob[b], best[b]);
      if (has2) best2 = group_best(g, o2, best2);
      // rows with more than 64 * kHeld listed pixels in the tile: one key update per group
      for (int e = (int)lane + kWave * kHeld; e < cnt; e += kWave) {
        int o, slot;
        if constexpr (kSorted) { o = (int)(idx_at(e0 + e) - rowbase); slot = e0 + e; }
        else { o = sm.eo[e]; slot = sm.es[e]; }
        key_min(slot, group_best(g, o, 0xFFFFFFFFu));
      }
      wave_lds_order();   // LDS free for the next group / row
    }
    pend_best2 = best2;
#pragma unroll
    for (int b = 0; b < NB; ++b) pend_best[b] = best[b];
    if constexpr (kSorted) { pend_e0 = e0; pend_cnt = cnt; }
    else pend_slot = has[0] ? slot0 : -1;
  };

  // Walk down the rows. The loads for the step y -> y + 1 (padded row
  // y + 2r + 1 enters the window, padded row y leaves it) are issued one step
  // ahead; the copies hold one spare padded row (and the image rows are
  // clamped) so the last, unused prefetch stays in bounds.
  int qin = ya + 2 * r + 1, qout = ya;
  const uint32_t* rin = rp0 + (int64_t)qin * rpw;
  const uint32_t* rout = rp0 + (int64_t)qout * rpw;
  RowRegs<DC, COLS> En, Ex;
  load_row<DC, COLS>(ls.row(qin), ls, rin, lo, En);
  load_row<DC, COLS>(ls.row(qout), ls, rout, lo, Ex);
  // Row ya (active by construction), then the steps y = ya + 1 .. yb. A
  // step takes its row's listed pixels (loaded a full step earlier) before it
  // issues the next step's loads, so the only waits are the slide's and a
  // short one for that list data.
  take_row(ya);
  int ynext = next_active(ya);   // the next active row (-1: none)
  load_next(ynext);
  pin_step(acc.v);
  entries_row(ya);
  for (int y = ya + 1; y <= yb; ++y) {
    const bool act = y == ynext;
    pin_step(acc.v);
    slide_row<DC, kPack, COLS>(En, Ex, acc, ls);
    pin_step(acc.v);
    flush();
    if (act) take_row(y);
    ++qin; ++qout; rin += rpw; rout += rpw;
    load_row<DC, COLS>(ls.row(qin), ls, rin, lo, En);
    load_row<DC, COLS>(ls.row(qout), ls, rout, lo, Ex);
    if (act) {
      ynext = next_active(y);
      load_next(ynext);
      pin_step(acc.v);
      entries_row(y);
    }
  }
  flush();
}

// Ordered and unordered lists, packed and 32-bit accumulators take separate
// instances (fewer live registers in each).
// 16-disparity chunks exist only with packed accumulators (the host uses
// 8-disparity chunks for frames whose window sums need 32 bits).
template <bool kPack>
__device__ __forceinline__ void tile_item8(const FrameDev& f, int tile, int chunk8, bool unsorted, int xs, int xe,
                                           TileLds& sm) {
  if (unsorted) tile_item_impl<8, false, kPack, 4>(f, tile, chunk8, xs, xe, sm);
  else tile_item_impl<8, true, kPack, 4>(f, tile, chunk8, xs, xe, sm);
}

// The same as an out-of-line call: inside the 16-disparity kernels its
// registers then do not add to those of the 16-disparity instance (it serves
// the less common frames there).
template <bool kPack>
__device__ __noinline__ void tile_item8_call(const FrameDev& f, int tile, int chunk8, bool unsorted, int xs, int xe,
                                             TileLds& sm) {
  tile_item8<kPack>(f, tile, chunk8, unsorted, xs, xe, sm);
}

// Items of a launch that has frames laid out with 8 columns per lane, other
// than ordered lists of such frames: unordered lists of those frames run the
// 4-column instance in passes of at most the 4-column width; frames with 4
// columns per lane run the 8-disparity 4-column instances. Out of line, so
// the wide instance's registers stay its own.
__device__ __noinline__ void tile_item_wide_rest(const FrameDev& f, int tile, int chunk8, bool unsorted, int x0, int x1,
                                                 TileLds& sm) {
  if (f.cpl == 8) {
    const int w4 = (Geom<4>::kSpanC - f.lpad - f.r) & ~3;
#pragma unroll 1
    for (int xs = x0; xs < x1; xs += w4) tile_item_impl<8, false, true, 4>(f, tile, chunk8, xs, min(xs + w4, x1), sm);
    return;
  }
  if (f.pack) tile_item8<true>(f, tile, chunk8, unsorted, x0, x1, sm);
  else tile_item8<false>(f, tile, chunk8, unsorted, x0, x1, sm);
}

// Dispatch of one work item. kWide launches (8-disparity chunks, some frames
// laid out with 8 columns per lane): ordered lists of those frames run the
// wide instance, everything else tile_item_wide_rest. Other launches (every
// frame with 4 columns per lane): a 16-disparity item of an ordered list with
// packed accumulators runs as one pass; any other frame runs its 16
// disparities as two 8-disparity passes (same work decomposition, fewer
// registers).
template <int DC, bool kWide>
__device__ __forceinline__ void tile_item(const FrameDev& f, int tile, int chunk, TileLds& sm) {
  const bool unsorted = *(g_uint32*)f.state & kUnsorted;
  const int x0 = (tile % f.ntx) * f.txo, x1 = min(x0 + f.txo, f.W);
  if constexpr (kWide) {
    static_assert(DC == 8, "wide launches use 8-disparity chunks");
    if (f.cpl == 8 && !unsorted) tile_item_impl<8, true, true, 8>(f, tile, chunk, x0, x1, sm);
    else tile_item_wide_rest(f, tile, chunk, unsorted, x0, x1, sm);
    return;
  }
  if (DC == 16 && f.pack && !unsorted) {
    tile_item_impl<16, true, true, 4>(f, tile, chunk, x0, x1, sm);
    return;
  }
  constexpr int kParts = DC / 8;
#pragma unroll 1
  for (int h = 0; h < kParts; ++h) {
    const int c8 = kParts * chunk + h;
    if (c8 * 8 > f.dmax) break;
    if constexpr (DC == 8) {
      if (f.pack) tile_item8<true>(f, tile, c8, unsorted, x0, x1, sm);
      else tile_item8<false>(f, tile, c8, unsorted, x0, x1, sm);
    } else {
      if (f.pack) tile_item8_call<true>(f, tile, c8, unsorted, x0, x1, sm);
      else tile_item8_call<false>(f, tile, c8, unsorted, x0, x1, sm);
    }
  }
}

// Occupancy target: four wavefronts per SIMD (128 VGPRs); three (168 VGPRs)
// for wide launches, whose 8-column instance needs the registers.
template <int DC, bool kWide>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWide ? 3 : 4, 8))) void k_tile_grid(
    const FrameDev* __restrict__ table, int fi) {
  __shared__ TileLds sm;
  const FrameDev& f = table[fi];
  const uint32_t item = blockIdx.x;
  tile_item<DC, kWide>(f, (int)(item / (uint32_t)f.nch), (int)(item % (uint32_t)f.nch), sm);
}

// Persistent form: one work queue per XCD. Tile t of a frame goes to queue
// t % 8, so the disparity chunks of a tile run on one XCD and share its L2.
// Workgroup w starts on queue w % 8 (the XCD the hardware places it on) and,
// once that queue is empty, takes items from the others.
template <int DC, bool kWide>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWide ? 3 : 4, 8))) void k_tile_persistent(
    const FrameDev* __restrict__ table, int nframes, QueueTotals totals, WsHeader* hdr) {
  __shared__ TileLds sm;
  __shared__ long long next_item;
  const int home = blockIdx.x % kQueues;
  for (int qi = 0; qi < kQueues; ++qi) {
    const int q = (home + qi) % kQueues;
    const int64_t total = totals.t[q];
    for (;;) {
      if (threadIdx.x == 0) next_item = (long long)atomicAdd(&hdr->q[q].head, 1ull);
      __syncthreads();
      // the same for every lane: read as a scalar, so the frame lookup and the
      // descriptor loads below stay scalar
      const uint64_t itv = (uint64_t)next_item;
      const int64_t it = (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(itv >> 32)) << 32) |
                                   (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)itv));
      __syncthreads();
      if (it >= total) break;
      // frame of this item: last frame with xbase[q] <= it
      int lo = 0, hi = nframes - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].xbase[q] <= it) lo = mid; else hi = mid - 1;
      }
      const FrameDev& f = table[lo];
      const uint32_t local = (uint32_t)(it - f.xbase[q]);
      const int tile = q + kQueues * (int)(local / (uint32_t)f.nch);
      tile_item<DC, kWide>(f, tile, (int)(local % (uint32_t)f.nch), sm);
    }
  }
}

// Keys split into (disparity, cost), four entries per thread and step. An
// ordered list holds its indices >= W*H in a tail from the first such slot on
// (k_check recorded it and answered those entries): the entries before it
// take key k, and the list itself is not read again. An unordered list
// reads each index for its representative slot. One 4-byte store of
// disparities and one 16-byte store of costs where the caller's arrays allow
// them (out_disp 4-byte, out_cost 16-byte aligned; for unordered lists also
// idx 16-byte aligned).
__global__ __launch_bounds__(256) void k_finalize(const FrameDev* __restrict__ table, int f0) {
  const FrameDev& f = table[f0 + blockIdx.y];
  const int64_t N = (int64_t)f.W * f.H;
  const bool unsorted = (*f.state & kUnsorted) != 0;
  const int64_t n = unsorted ? f.n : min(f.n, (int64_t)*(const uint64_t*)(f.state + 2));
  const uint32_t* idx = f.idx;
  const uint32_t* keys = f.keys;
  uint8_t* od = f.out_disp;
  uint32_t* oc = f.out_cost;
  const bool vec = ((uintptr_t)od & 3u) == 0 && ((uintptr_t)oc & 15u) == 0 &&
                   (!unsorted || ((uintptr_t)idx & 15u) == 0);
  for (int64_t k = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x); k < n; k += 4 * (int64_t)gridDim.x * blockDim.x) {
    if (vec && k + 3 < n) {
      uint32_t key[4];
      bool out[4] = {false, false, false, false};
      if (!unsorted) {
        const u32x4 kv = *(g_uint4*)(keys + k);
        key[0] = kv.x; key[1] = kv.y; key[2] = kv.z; key[3] = kv.w;
      } else {
        const u32x4 v = *(g_uint4*)(idx + k);
        const uint32_t p[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          out[j] = (int64_t)p[j] >= N;   // (255, ~0) as k_check wrote them
          key[j] = out[j] ? 0u : keys[f.map[p[j]]];
        }
      }
      uint32_t cost[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cost[j] = out[j] ? 0xFFFFFFFFu : key[j] >> 8;
        key[j] = out[j] ? 0xFFu : key[j] & 0xFFu;
      }
      *(__attribute__((address_space(1))) uint32_t*)(od + k) = key[0] | (key[1] << 8) | (key[2] << 16) | (key[3] << 24);
      if (oc) *(g_uint4_rw*)(oc + k) = u32x4{cost[0], cost[1], cost[2], cost[3]};
      continue;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (k + j >= n) break;
      int64_t slot = k + j;
      if (unsorted) {
        const uint32_t p = idx[k + j];
        if ((int64_t)p >= N) continue;
        slot = f.map[p];
      }
      const uint32_t key = keys[slot];
      od[k + j] = (uint8_t)(key & 0xFFu);
      if (oc) oc[k + j] = key >> 8;
    }
  }
}

// ---------------------------------------------------------------------------
// Reference: one wavefront per list entry, lanes over disparities, direct
// clamped reads of the original images.
__global__ __launch_bounds__(256) void k_ref(const uint8_t* __restrict__ L, const uint8_t* __restrict__ R,
                                             int W, int H, int C, int64_t pitch,
                                             const uint32_t* __restrict__ idx, int64_t n, int r, int dmax,
                                             uint8_t* od, uint32_t* oc, uint32_t* err) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); k < n; k += nw) {
    const uint32_t p = idx[k];
    if ((int64_t)p >= (int64_t)W * H) {
      if (lane == 0) {
        od[k] = 255;
        if (oc) oc[k] = 0xFFFFFFFFu;
        if (err) atomicOr(err, 1u);
      }
      continue;
    }
    const int x = (int)(p % (uint32_t)W), y = (int)(p / (uint32_t)W);
    uint32_t best = 0xFFFFFFFFu;
    for (int d = lane; d <= dmax; d += 64) {
      uint32_t s = 0;
      for (int j = -r; j <= r; ++j) {
        const int yy = clampi(y + j, 0, H - 1);
        const uint8_t* lr = L + (int64_t)yy * pitch;
        const uint8_t* rr = R + (int64_t)yy * pitch;
        for (int i = -r; i <= r; ++i) {
          const uint8_t* a = lr + (int64_t)clampi(x + i, 0, W - 1) * C;
          const uint8_t* b = rr + (int64_t)clampi(x - d + i, 0, W - 1) * C;
          for (int c = 0; c < C; ++c) s += (uint32_t)abs((int)a[c] - (int)b[c]);
        }
      }
      best = min(best, (s << 8) | (uint32_t)d);
    }
    for (int off = 32; off >= 1; off >>= 1) best = min(best, (uint32_t)__shfl_xor((int)best, off, 64));
    if (lane == 0) {
      od[k] = (uint8_t)(best & 0xFFu);
      if (oc) oc[k] = best >> 8;
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side launch helpers (called from sbs_api.hip).
hipError_t launch_put_desc(FrameDev* table, const FrameDev* host, int nframes, hipStream_t s) {
  for (int first = 0; first < nframes; first += kDescPerLaunch) {
    DescBatch b{};
    b.first = first;
    b.count = nframes - first < kDescPerLaunch ? nframes - first : kDescPerLaunch;
    for (int i = 0; i < b.count; ++i) b.f[i] = host[first + i];
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(kDescPerLaunch), 0, s, table, b);
  }
  return hipGetLastError();
}

// Blocks per frame of the list kernels (grid-stride over the list): 64 fill
// the chip when a launch covers many frames; fewer frames per launch take
// more each, so that a single frame's list is not walked by 64 blocks alone.
int list_blocks(int nf) { return nf >= 32 ? 64 : 2048 / nf; }

hipError_t launch_prologue(const FrameDev* table, int f0, int nf, int max_rows, WsHeader* hdr,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_check, dim3(list_blocks(nf), nf), dim3(256), 0, s, table, f0, hdr);
  int gx = max_rows < 2048 ? max_rows : 2048;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_prep, dim3(gx, nf), dim3(256), 0, s, table, f0);
  hipLaunchKernelGGL(k_scatter, dim3(256, nf), dim3(256), 0, s, table, f0);
  return hipGetLastError();
}

hipError_t launch_finalize(const FrameDev* table, int f0, int nf, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(list_blocks(nf), nf), dim3(256), 0, s, table, f0);
  return hipGetLastError();
}

hipError_t launch_tile_grid(const FrameDev* table, int fi, int64_t nitems, int chunk, bool wide, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const dim3 g((unsigned)nitems), b(64);
  if (wide) hipLaunchKernelGGL((k_tile_grid<8, true>), g, b, 0, s, table, fi);
  else if (chunk == 8) hipLaunchKernelGGL((k_tile_grid<8, false>), g, b, 0, s, table, fi);
  else hipLaunchKernelGGL((k_tile_grid<16, false>), g, b, 0, s, table, fi);
  return hipGetLastError();
}

hipError_t launch_tile_persistent(const FrameDev* table, int nframes, const QueueTotals& totals, int chunk, bool wide,
                                  int grid, WsHeader* hdr, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_head, dim3(1), dim3(64), 0, s, hdr);
  const dim3 g(grid), b(64);
  if (wide) hipLaunchKernelGGL((k_tile_persistent<8, true>), g, b, 0, s, table, nframes, totals, hdr);
  else if (chunk == 8) hipLaunchKernelGGL((k_tile_persistent<8, false>), g, b, 0, s, table, nframes, totals, hdr);
  else hipLaunchKernelGGL((k_tile_persistent<16, false>), g, b, 0, s, table, nframes, totals, hdr);
  return hipGetLastError();
}

hipError_t launch_ref(const uint8_t* L, const uint8_t* R, int W, int H, int C, int64_t pitch, const uint32_t* idx,
                      int64_t n, int r, int dmax, uint8_t* od, uint32_t* oc, uint32_t* err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_ref, dim3((unsigned)blocks), dim3(256), 0, s, L, R, W, H, C, pitch, idx, n, r, dmax, od, oc,
                     err);
  return hipGetLastError();
}

}  // namespace sbs
