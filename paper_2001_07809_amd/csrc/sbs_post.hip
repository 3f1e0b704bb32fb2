// Steps after the disparity search (arXiv 2001.07809, Sec. III):
//   * disparity map reconstruction from the listed pixels' disparities:
//     Algorithm 1 (fill along scan lines), then Algorithm 2 (peek along
//     columns at the nearest determined pixels above and below);
//   * depth-based selective blurring with the normalised Gaussian of Eq. 1-2.
// Declared in include/sbs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <utility>

#include "../../include/sbs.h"
#include "sbs_internal.h"

namespace sbs_post {

constexpr int kRowThreads = 256;

// slot[p] = largest list position k with idx[k] == p (so a repeated index keeps its last value).
__global__ __launch_bounds__(256) void k_rc_clear(int32_t* slot, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    slot[i] = -1;
}

// In two passes without an atomic per entry: every entry stores its
// position (an entry followed by one of the same index leaves it to that
// one), so a pixel holds one of its positions; then every entry whose
// position is above what its pixel holds raises it with an atomic maximum,
// which leaves the largest (only repeats that are not adjacent need one).
__global__ __launch_bounds__(256) void k_rc_scatter(const uint32_t* idx, int64_t n, int64_t N, int32_t* slot) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = idx[k];
    if ((int64_t)p < N && (k + 1 == n || idx[k + 1] != p)) slot[p] = (int32_t)k;
  }
}
__global__ __launch_bounds__(256) void k_rc_scatter_max(const uint32_t* idx, int64_t n, int64_t N, int32_t* slot) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = idx[k];
    if ((int64_t)p < N && slot[p] < (int32_t)k) atomicMax(&slot[p], (int32_t)k);
  }
}

// Algorithm 1, one block of four wavefronts per row: a pixel strictly
// between two consecutive listed pixels of the row that carry the same
// disparity takes it. Each wavefront owns a quarter of the row's 64-pixel
// chunks and walks them one pixel per lane (coalesced): a ballot marks a
// chunk's listed pixels, the nearest one at or left of each lane comes from
// the mask's bits up to the lane (its value by a lane shuffle), and the last
// listed value of the chunks before is carried as a wave-uniform value. A
// left-to-right pass writes, per pixel, the value of the nearest listed pixel
// on its left within the quarter (-2: none there yet) and records the
// quarter's first and last listed values; after an exchange through LDS a
// right-to-left pass finds the nearest listed pixel on the right the same
// way, takes the one on the left from the quarters before where it was
// missing, and decides. Output: f[p] = disparity or -1 (undetermined).
constexpr int kFillChunks = 16;   // 64-pixel chunks per quarter held in registers (rows up to 4096 pixels)
__global__ __launch_bounds__(kRowThreads) void k_rc_fill(const int32_t* slot, const uint8_t* disp, int32_t W,
                                                           int32_t H, int16_t* f) {
  constexpr int kWaves = kRowThreads / 64;
  __shared__ int q_first[kWaves], q_last[kWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nch = (W + 63) >> 6, per = (nch + kWaves - 1) / kWaves;
  const int c0 = min(wv * per, nch), c1 = min(c0 + per, nch);
  const uint64_t upto = (2ull << lane) - 1ull;    // bits 0 .. lane
  const uint64_t from = ~((1ull << lane) - 1ull); // bits lane .. 63
  if (per <= kFillChunks) {
    // a quarter of at most kFillChunks chunks: its slots are loaded at once,
    // then its disparities, and both passes run on registers (one round trip
    // to memory for each, and the row is written once)
    for (int y = blockIdx.x; y < H; y += gridDim.x) {
      const int32_t* srow = slot + (int64_t)y * W;
      int16_t* frow = f + (int64_t)y * W;
      int v[kFillChunks];
#pragma unroll
      for (int i = 0; i < kFillChunks; ++i) {
        const int x = ((c0 + i) << 6) + lane;
        v[i] = (c0 + i < c1 && x < W) ? srow[x] : -1;   // slot here, disparity below
      }
#pragma unroll
      for (int i = 0; i < kFillChunks; ++i) v[i] = v[i] >= 0 ? (int)disp[v[i]] : -1;
      int lft[kFillChunks];   // nearest listed value at or left of the pixel within the quarter, -2: none
      int carry = -2, first = -1;
#pragma unroll
      for (int i = 0; i < kFillChunks; ++i) {
        const uint64_t m = __builtin_amdgcn_ballot_w64(v[i] >= 0);
        const uint64_t b = m & upto;
        const int left = __shfl(v[i], b ? 63 - __builtin_clzll(b) : 0);
        lft[i] = b ? left : carry;
        if (m) {
          if (first < 0) first = __shfl(v[i], __builtin_ctzll(m));
          carry = __shfl(v[i], 63 - __builtin_clzll(m));
        }
      }
      if (lane == 0) { q_first[wv] = first; q_last[wv] = carry < 0 ? -1 : carry; }
      __syncthreads();
      int cl = -1, cr = -1;   // nearest listed value in the quarters to the left / right
      for (int j = wv - 1; j >= 0 && cl < 0; --j) cl = q_last[j];
      for (int j = wv + 1; j < kWaves && cr < 0; ++j) cr = q_first[j];
      __syncthreads();   // the next row rewrites q_first / q_last
      carry = cr;
#pragma unroll
      for (int i = kFillChunks - 1; i >= 0; --i) {
        const int x = ((c0 + i) << 6) + lane;
        const uint64_t m = __builtin_amdgcn_ballot_w64(v[i] >= 0);
        const uint64_t b = m & from;
        const int right = b ? __shfl(v[i], __builtin_ctzll(b)) : carry;
        if (c0 + i < c1 && x < W) {
          int left = lft[i];
          if (left == -2) left = cl;
          frow[x] = (int16_t)(v[i] >= 0 ? v[i] : ((left >= 0 && left == right) ? left : -1));
        }
        if (m) carry = __shfl(v[i], __builtin_ctzll(m));
      }
    }
    return;
  }
  for (int y = blockIdx.x; y < H; y += gridDim.x) {
    const int32_t* srow = slot + (int64_t)y * W;
    int16_t* frow = f + (int64_t)y * W;
    int carry = -2, first = -1;
#pragma unroll 4
    for (int c = c0; c < c1; ++c) {
      const int x = (c << 6) + lane;
      const int32_t k = x < W ? srow[x] : -1;
      const int v = k >= 0 ? (int)disp[k] : -1;
      const uint64_t m = __builtin_amdgcn_ballot_w64(k >= 0);
      const uint64_t b = m & upto;
      const int left = __shfl(v, b ? 63 - __builtin_clzll(b) : 0);
      if (x < W) frow[x] = (int16_t)(b ? left : carry);
      if (m) {
        if (first < 0) first = __shfl(v, __builtin_ctzll(m));
        carry = __shfl(v, 63 - __builtin_clzll(m));
      }
    }
    if (lane == 0) { q_first[wv] = first; q_last[wv] = carry < 0 ? -1 : carry; }
    __syncthreads();
    int cl = -1, cr = -1;   // nearest listed value in the quarters to the left / right
    for (int j = wv - 1; j >= 0 && cl < 0; --j) cl = q_last[j];
    for (int j = wv + 1; j < kWaves && cr < 0; ++j) cr = q_first[j];
    __syncthreads();   // the next row rewrites q_first / q_last
    carry = cr;
#pragma unroll 4
    for (int c = c1 - 1; c >= c0; --c) {
      const int x = (c << 6) + lane;
      const int32_t k = x < W ? srow[x] : -1;
      const int v = k >= 0 ? (int)disp[k] : -1;
      const uint64_t m = __builtin_amdgcn_ballot_w64(k >= 0);
      const uint64_t b = m & from;
      const int right = b ? __shfl(v, __builtin_ctzll(b)) : carry;
      if (x < W) {
        int left = frow[x];
        if (left == -2) left = cl;
        frow[x] = (int16_t)(k >= 0 ? v : ((left >= 0 && left == right) ? left : -1));
      }
      if (m) carry = __shfl(v, __builtin_ctzll(m));
    }
  }
}

// Algorithm 2: an undetermined pixel takes the smaller of its nearest
// determined pixels above and below when their range exceeds the threshold,
// else their mean rounded half up; one-sided when only one exists; 0 when the
// column has none. Reads only Algorithm 1's output, so every column is
// independent. A column is cut into segments of `seglen` rows (16: many
// short walks fill the chip better than fewer long ones; more for images
// over 1M rows so the segments fit the grid), one thread per
// (column, segment): k_rc_colseg records each segment's topmost and
// bottommost determined value, k_rc_chunks / k_rc_colscan / k_rc_segscan
// turn those records into the nearest determined value above and below each
// segment (scans down and up each column over chunk summaries, so a column
// with few determined pixels costs O(nseg), not O(nseg^2)), and k_rc_peek
// resolves the segment's rows in two passes
// (threads of a block cover adjacent columns, so every row access is
// coalesced).
constexpr int kColSeg = 16;

__global__ __launch_bounds__(256) void k_rc_colseg(const int16_t* f, int32_t W, int32_t H, int32_t seglen,
                                                   int16_t* seg_first, int16_t* seg_last) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int sg = blockIdx.y;
  if (x >= W) return;
  const int y0 = sg * seglen, y1 = min(y0 + seglen, H);
  int16_t first = -1, last = -1;
  if (seglen == kColSeg) {
    // the segment's values read at once
    int16_t v[kColSeg];
#pragma unroll
    for (int k = 0; k < kColSeg; ++k) v[k] = y0 + k < y1 ? f[(int64_t)(y0 + k) * W + x] : (int16_t)-1;
#pragma unroll
    for (int k = 0; k < kColSeg; ++k)
      if (v[k] >= 0) {
        if (first < 0) first = v[k];
        last = v[k];
      }
  } else {
    for (int y = y0; y < y1; ++y) {
      const int16_t v = f[(int64_t)y * W + x];
      if (v >= 0) {
        if (first < 0) first = v;
        last = v;
      }
    }
  }
  seg_first[(int64_t)sg * W + x] = first;
  seg_last[(int64_t)sg * W + x] = last;
}

// In place: seg_last[sg] becomes the nearest determined value above segment
// sg (the last one of the segments before it), seg_first[sg] the nearest
// below it (the first one of the segments after it); -1 where none. Three
// launches over chunks of kScanBatch segments: k_rc_chunks sums up each
// chunk (its last and first determined value; one thread per column and
// chunk), k_rc_colscan turns the summaries into the same nearest values per
// chunk (one thread per column, a pass down and one up, kScanBatch records
// in flight), and k_rc_segscan rewrites each chunk's records from its
// chunk's carries (one thread per column and chunk). A column's sequential
// work is its chunk count, a sixteenth of its segment count.
constexpr int kScanBatch = 16;
__global__ __launch_bounds__(256) void k_rc_chunks(int32_t W, int32_t nseg, const int16_t* seg_first,
                                                   const int16_t* seg_last, int16_t* ch_first, int16_t* ch_last) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (x >= W) return;
  const int s0 = c * kScanBatch;
  int16_t vl[kScanBatch], vf[kScanBatch];
#pragma unroll
  for (int k = 0; k < kScanBatch; ++k) {
    const bool in = s0 + k < nseg;
    vl[k] = in ? seg_last[(int64_t)(s0 + k) * W + x] : (int16_t)-1;
    vf[k] = in ? seg_first[(int64_t)(s0 + k) * W + x] : (int16_t)-1;
  }
  int16_t last = -1, first = -1;
#pragma unroll
  for (int k = 0; k < kScanBatch; ++k) {
    if (vl[k] >= 0) last = vl[k];
    if (first < 0 && vf[k] >= 0) first = vf[k];
  }
  ch_last[(int64_t)c * W + x] = last;
  ch_first[(int64_t)c * W + x] = first;
}

// In place over n records of each column: last[i] becomes the last
// non-negative value of records 0 .. i - 1, first[i] the first of records
// i + 1 .. n - 1 (-1 where none). Records are read kScanBatch at a time
// before any of them is written.
__global__ __launch_bounds__(256) void k_rc_colscan(int32_t W, int32_t n, int16_t* first, int16_t* last) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= W) return;
  int16_t carry = -1;
  for (int s0 = 0; s0 < n; s0 += kScanBatch) {
    int16_t v[kScanBatch];
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) v[k] = s0 + k < n ? last[(int64_t)(s0 + k) * W + x] : (int16_t)-1;
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) {
      if (s0 + k >= n) break;
      last[(int64_t)(s0 + k) * W + x] = carry;
      if (v[k] >= 0) carry = v[k];
    }
  }
  carry = -1;
  for (int s1 = n - 1; s1 >= 0; s1 -= kScanBatch) {   // records s1, s1 - 1, ...
    int16_t v[kScanBatch];
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) v[k] = s1 - k >= 0 ? first[(int64_t)(s1 - k) * W + x] : (int16_t)-1;
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) {
      if (s1 - k < 0) break;
      first[(int64_t)(s1 - k) * W + x] = carry;
      if (v[k] >= 0) carry = v[k];
    }
  }
}

__global__ __launch_bounds__(256) void k_rc_segscan(int32_t W, int32_t nseg, int16_t* seg_first, int16_t* seg_last,
                                                    const int16_t* ch_first, const int16_t* ch_last) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (x >= W) return;
  const int s0 = c * kScanBatch;
  int16_t vl[kScanBatch], vf[kScanBatch];
#pragma unroll
  for (int k = 0; k < kScanBatch; ++k) {
    const bool in = s0 + k < nseg;
    vl[k] = in ? seg_last[(int64_t)(s0 + k) * W + x] : (int16_t)-1;
    vf[k] = in ? seg_first[(int64_t)(s0 + k) * W + x] : (int16_t)-1;
  }
  // the last determined value of the chunks before this one, the first of
  // those after it (one chunk: none)
  int16_t above = gridDim.y > 1 ? ch_last[(int64_t)c * W + x] : (int16_t)-1;
  int16_t below = gridDim.y > 1 ? ch_first[(int64_t)c * W + x] : (int16_t)-1;
#pragma unroll
  for (int k = 0; k < kScanBatch; ++k) {
    if (s0 + k >= nseg) break;
    seg_last[(int64_t)(s0 + k) * W + x] = above;
    if (vl[k] >= 0) above = vl[k];
  }
#pragma unroll
  for (int k = kScanBatch - 1; k >= 0; --k) {
    if (s0 + k >= nseg) continue;
    seg_first[(int64_t)(s0 + k) * W + x] = below;
    if (vf[k] >= 0) below = vf[k];
  }
}

__global__ __launch_bounds__(256) void k_rc_peek(const int16_t* f, int32_t W, int32_t H, int32_t threshold,
                                                 int32_t seglen, const int16_t* above_seg, const int16_t* below_seg,
                                                 int16_t* up, uint8_t* out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int sg = blockIdx.y;
  if (x >= W) return;
  const int y0 = sg * seglen, y1 = min(y0 + seglen, H);
  // nearest determined value above the segment, and below it (k_rc_segscan)
  int16_t last = above_seg[(int64_t)sg * W + x];
  int16_t below = below_seg[(int64_t)sg * W + x];
  auto resolve = [&](int a, int b) -> uint8_t {
    int r;
    if (a < 0 && b < 0) r = 0;
    else if (a < 0) r = b;
    else if (b < 0) r = a;
    else if (abs(a - b) > threshold) r = min(a, b);
    else r = (a + b + 1) / 2;
    return (uint8_t)r;
  };
  if (seglen == kColSeg) {
    // the segment's values read at once, the nearest value above each row
    // kept in registers
    int16_t v[kColSeg], a[kColSeg];
#pragma unroll
    for (int k = 0; k < kColSeg; ++k) v[k] = y0 + k < y1 ? f[(int64_t)(y0 + k) * W + x] : (int16_t)-1;
#pragma unroll
    for (int k = 0; k < kColSeg; ++k) {
      a[k] = last;
      if (v[k] >= 0) last = v[k];
    }
#pragma unroll
    for (int k = kColSeg - 1; k >= 0; --k) {
      if (y0 + k >= y1) continue;
      uint8_t r;
      if (v[k] >= 0) { r = (uint8_t)v[k]; below = v[k]; }
      else r = resolve(a[k], below);
      out[(int64_t)(y0 + k) * W + x] = r;
    }
    return;
  }
  for (int y = y0; y < y1; ++y) {
    const int16_t v = f[(int64_t)y * W + x];
    up[(int64_t)y * W + x] = last;
    if (v >= 0) last = v;
  }
  for (int y = y1 - 1; y >= y0; --y) {
    const int64_t q = (int64_t)y * W + x;
    const int16_t v = f[q];
    if (v >= 0) {
      out[q] = (uint8_t)v;
      below = v;
      continue;
    }
    out[q] = resolve(up[q], below);
  }
}

// Selective blur: separable Gaussian (normalised per axis, so the product is
// Eq. 2's normalised 2-D kernel), replicate border, fp32 accumulation.
constexpr int kMaxRadius = 64;
constexpr int kMaxRanges = 16;

struct BlurArgs {
  float g[2 * kMaxRadius + 1];
  int32_t lo[kMaxRanges], hi[kMaxRanges];
  int32_t rad, nranges;
};

// One thread per pixel and all its channels (pixel indices are below 2^31,
// so the row and column come from 32-bit division).
__global__ __launch_bounds__(256) void k_blur_h(const uint8_t* img, int32_t W, int32_t H, int32_t C, int64_t pitch,
                                                BlurArgs a, float* tmp) {
  const int64_t N = (int64_t)W * H;
  for (int64_t px = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; px < N; px += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)((uint32_t)px % (uint32_t)W), y = (int)((uint32_t)px / (uint32_t)W);
    const uint8_t* row = img + (int64_t)y * pitch;
    for (int c = 0; c < C; ++c) {
      float s = 0.f;
      for (int k = -a.rad; k <= a.rad; ++k) {
        const int xx = min(max(x + k, 0), W - 1);
        s += a.g[k + a.rad] * (float)row[(int64_t)xx * C + c];
      }
      tmp[px * C + c] = s;
    }
  }
}

__global__ __launch_bounds__(256) void k_blur_v(const uint8_t* img, const uint8_t* depth, int32_t W, int32_t H,
                                                int32_t C, int64_t pitch, BlurArgs a, const float* tmp, float* out) {
  const int64_t N = (int64_t)W * H;
  for (int64_t px = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; px < N; px += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)((uint32_t)px % (uint32_t)W), y = (int)((uint32_t)px / (uint32_t)W);
    const int dv = depth[px];
    bool keep = false;
    for (int t = 0; t < a.nranges; ++t) keep |= (dv >= a.lo[t] && dv <= a.hi[t]);
    if (keep) {
      for (int c = 0; c < C; ++c) out[px * C + c] = (float)img[(int64_t)y * pitch + (int64_t)x * C + c];
      continue;
    }
    for (int c = 0; c < C; ++c) {
      float s = 0.f;
      for (int k = -a.rad; k <= a.rad; ++k) {
        const int yy = min(max(y + k, 0), H - 1);
        s += a.g[k + a.rad] * tmp[((int64_t)yy * W + x) * C + c];
      }
      out[px * C + c] = s;
    }
  }
}

// The same blur in one pass per tile of kBlurTX x kBlurTY pixels (radius up
// to kBlurTileRad, a compile-time constant per instance so the tap loops
// unroll):
//  - the tile's in-focus flags first: a tile whose every pixel is in focus
//    only converts its pixels (no input tile, no sums);
//  - the clamped input rows and columns go to LDS, as aligned dword loads
//    where the image rows start on 4-byte boundaries and the tile does not
//    reach past a side edge, byte by byte with clamped columns otherwise;
//  - the horizontal pass runs over the tile's rows plus the vertical halo,
//    each thread 8 adjacent outputs of one row and channel from 8 + 2 RAD
//    input bytes (lanes over rows and channels: no LDS bank conflicts), into
//    an LDS float tile with padded rows;
//  - the vertical pass, each thread 8 rows of one column and channel from
//    8 + 2 RAD horizontal sums (lanes over columns: coalesced stores).
// Each sum runs over the taps in the same order as in the two kernels
// above, so the results are the same floats; the intermediate image never
// travels through HBM.
constexpr int kBlurTX = 64, kBlurTY = 32, kBlurTileRad = 14;
constexpr int kBlurRun = 8;   // outputs per thread and pass
constexpr int kBlurThreads = 512;   // eight wavefronts per tile: 24 per CU at three tiles

template <int C, int RAD>
struct BlurTileGeom {
  static constexpr int rows = kBlurTY + 2 * RAD;              // image rows y0 - RAD ..
  static constexpr int cols = kBlurTX + 2 * RAD;              // image columns x0 - RAD ..
  static constexpr int rowb = cols * C;                       // input bytes per row
  static constexpr int rowbp = (rowb + 3) & ~3;
  static constexpr int hrow = kBlurTX * C + 1;                // floats per horizontal-sum row (padded)
  static constexpr size_t lds = (size_t)rows * hrow * 4 + (size_t)rows * rowbp + kBlurTX * kBlurTY;
};

template <int C, int RAD>
__global__ __launch_bounds__(kBlurThreads) void k_blur_tile(const uint8_t* img, const uint8_t* depth, int32_t W,
                                                            int32_t H, int64_t pitch, int32_t aligned, BlurArgs a,
                                                            float* out) {
  using G = BlurTileGeom<C, RAD>;
  extern __shared__ __attribute__((aligned(16))) unsigned char blur_lds[];
  float* hb = (float*)blur_lds;                                          // rows x hrow
  uint8_t* ib = blur_lds + (size_t)G::rows * G::hrow * 4;               // rows x rowbp input bytes
  uint8_t* keep = ib + (size_t)G::rows * G::rowbp;                       // kBlurTY x kBlurTX in-focus flags
  const int x0 = blockIdx.x * kBlurTX, y0 = blockIdx.y * kBlurTY;
  const int tid = threadIdx.x;

  // in-focus flags of the tile's pixels (1 outside the image: nothing to do there)
  bool need = false;
  for (int i = tid; i < kBlurTX * kBlurTY; i += kBlurThreads) {
    const int y = i / kBlurTX, x = i - y * kBlurTX;
    bool k = true;
    if (y0 + y < H && x0 + x < W) {
      const int dv = depth[(int64_t)(y0 + y) * W + x0 + x];
      k = false;
      for (int t = 0; t < a.nranges; ++t) k |= (dv >= a.lo[t] && dv <= a.hi[t]);
    }
    keep[i] = k ? 1 : 0;
    need |= !k;
  }
  if (!__syncthreads_or(need)) {
    // every pixel in focus: the image itself, as floats
    for (int i = tid; i < kBlurTY * kBlurTX * C; i += kBlurThreads) {
      const int y = i / (kBlurTX * C), xc = i - y * (kBlurTX * C);
      if (y0 + y < H && x0 * C + xc < W * C)
        out[((int64_t)(y0 + y) * W + x0) * C + xc] = (float)img[(int64_t)(y0 + y) * pitch + (int64_t)x0 * C + xc];
    }
    return;
  }

  // input tile: image rows y0 - RAD .. (clamped), columns x0 - RAD .. (clamped)
  if (aligned && x0 - RAD >= 0 && x0 + kBlurTX + RAD <= W) {
    const int s0 = (x0 - RAD) * C;                  // first byte of a tile row within its image row
    const int q0 = s0 & ~3;
    constexpr int ndw = (G::rowb + 3 + 3) / 4;      // dwords covering the row's bytes
    const int rowend = W * C;
    for (int i = tid; i < G::rows * ndw; i += kBlurThreads) {
      const int r = i / ndw, w = i - r * ndw;
      const int yy = min(max(y0 - RAD + r, 0), H - 1);
      const uint8_t* row = img + (int64_t)yy * pitch;
      const int q = q0 + 4 * w;
      uint32_t v = 0u;
      if (q + 3 < rowend) {
        v = *(const uint32_t*)(row + q);
      } else {
        for (int j = 0; j < 4; ++j)
          if (q + j < rowend) v |= (uint32_t)row[q + j] << (8 * j);
      }
      for (int j = 0; j < 4; ++j) {
        const int b = q + j - s0;
        if (b >= 0 && b < G::rowb) ib[r * G::rowbp + b] = (uint8_t)(v >> (8 * j));
      }
    }
  } else {
    for (int b = tid; b < G::rows * G::rowb; b += kBlurThreads) {
      const int r = b / G::rowb, jc = b - r * G::rowb, j = jc / C;
      const int yy = min(max(y0 - RAD + r, 0), H - 1), xx = min(max(x0 - RAD + j, 0), W - 1);
      ib[r * G::rowbp + jc] = img[(int64_t)yy * pitch + (int64_t)xx * C + (jc - j * C)];
    }
  }
  __syncthreads();

  // horizontal pass: item = (run of 8 columns, row, channel), rows and
  // channels varying fastest across lanes
  constexpr int hitems = (kBlurTX / kBlurRun) * G::rows * C;
  for (int i = tid; i < hitems; i += kBlurThreads) {
    const int run = i / (G::rows * C), rc = i - run * (G::rows * C);
    const int r = rc / C, c = rc - r * C;
    const uint8_t* src = ib + r * G::rowbp + run * kBlurRun * C + c;   // column run*8 + j - RAD at src[j * C]
    float v[kBlurRun + 2 * RAD];
#pragma unroll
    for (int j = 0; j < kBlurRun + 2 * RAD; ++j) v[j] = (float)src[j * C];
    float* dst = hb + r * G::hrow + run * kBlurRun * C + c;
#pragma unroll
    for (int o = 0; o < kBlurRun; ++o) {
      float s = 0.f;
#pragma unroll
      for (int k = -RAD; k <= RAD; ++k) s += a.g[k + RAD] * v[o + k + RAD];
      dst[o * C] = s;
    }
  }
  __syncthreads();

  // vertical pass: item = (run of 8 rows, column x channel), columns varying fastest
  constexpr int vitems = (kBlurTY / kBlurRun) * kBlurTX * C;
  for (int i = tid; i < vitems; i += kBlurThreads) {
    const int run = i / (kBlurTX * C), xc = i - run * (kBlurTX * C);
    const int x = xc / C;
    if (x0 + x >= W) continue;
    const float* col = hb + run * kBlurRun * G::hrow + xc;   // row run*8 + j - RAD (tile rows) at col[j * hrow]
    float v[kBlurRun + 2 * RAD];
#pragma unroll
    for (int j = 0; j < kBlurRun + 2 * RAD; ++j) v[j] = col[j * G::hrow];
#pragma unroll
    for (int o = 0; o < kBlurRun; ++o) {
      const int y = run * kBlurRun + o;
      if (y0 + y >= H) break;
      float s;
      if (keep[y * kBlurTX + x]) {
        s = (float)ib[(y + RAD) * G::rowbp + (x + RAD) * C + (xc - x * C)];
      } else {
        s = 0.f;
#pragma unroll
        for (int k = -RAD; k <= RAD; ++k) s += a.g[k + RAD] * v[o + k + RAD];
      }
      out[((int64_t)(y0 + y) * W + x0) * C + xc] = s;
    }
  }
}

template <int C, int RAD>
void launch_blur_tile(dim3 grid, hipStream_t s, const uint8_t* img, const uint8_t* depth, int32_t W, int32_t H,
                      int64_t pitch, int32_t aligned, const BlurArgs& a, float* out) {
  constexpr size_t lds = BlurTileGeom<C, RAD>::lds;
  hipLaunchKernelGGL((k_blur_tile<C, RAD>), grid, dim3(kBlurThreads), lds, s, img, depth, W, H, pitch, aligned, a,
                     out);
}

template <int C, int... R>
void blur_tile_dispatch(int rad, std::integer_sequence<int, R...>, dim3 grid, hipStream_t s, const uint8_t* img,
                        const uint8_t* depth, int32_t W, int32_t H, int64_t pitch, int32_t aligned, const BlurArgs& a,
                        float* out) {
  ((rad == R + 1 ? launch_blur_tile<C, R + 1>(grid, s, img, depth, W, H, pitch, aligned, a, out) : void()), ...);
}

// The same blur on the matrix cores, for radii up to 8 (sigma <= 2.67). At
// fp32 vector rates a 4096x2304 RGB frame's taps (13 + 13 per channel and
// pixel at sigma 2) take longer than its 151 MB take to cross HBM, so both
// tap passes run as 16x16x32 fp16 products with fp32 accumulation:
//  - horizontal: rows of the input tile (bytes, exact in fp16) times the
//    banded matrix of the taps, B[k][n] = g(k - n - (8 - radius));
//  - vertical: the same banded matrix times the horizontal sums.
// fp16 holds 11 significant bits, so the taps are split into a high and a
// low fp16 part (t = hi + lo, relative error ~2^-22) and so are the
// horizontal sums; the vertical pass adds hi*hi + lo*hi + hi*lo. The taps
// are scaled by 2^10 (exactly undone afterwards) so that their low parts are
// normal fp16 numbers. The products of the low parts are summed apart from
// the main ones, so their roundings stay small. Worst-case error against
// exact arithmetic: about 4e-4 on outputs in [0, 255] (per pass about 1e-4
// from the fp32 sums, 1.2e-4 from truncating the horizontal sums' low parts,
// 6e-5 for the low x low products left out).
// One tile of 64 x 32 outputs per workgroup of four wavefronts; wavefront w
// owns output columns 16w .. 16w + 15, so its horizontal sums feed only its
// own vertical pass (through its own LDS, in the order it issues them; no
// barrier). The input tile is 48 rows x 80 columns from image row y0 - 8 and
// column x0 - 8 (clamped), converted once to planar fp16.
typedef _Float16 h16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
typedef __fp16 fp16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int mu32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int mu32x3 __attribute__((ext_vector_type(3)));
typedef __attribute__((address_space(1))) const mu32x3 g_mu32x3;
typedef __attribute__((address_space(1))) const mu32x2 g_mu32x2;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 g_u32x4;
typedef __attribute__((address_space(1))) const uint32_t g_mu32;
typedef __attribute__((address_space(1))) mu32x3 g_mu32x3_rw;

constexpr int kMxTX = 64, kMxTY = 32;   // output tile
constexpr int kMxRad = 8;               // largest radius
constexpr int kMxRows = kMxTY + 2 * kMxRad, kMxCols = kMxTX + 2 * kMxRad;   // 48 x 80 input tile
constexpr int kMxPT = 56;               // fp16 per column of a wavefront's horizontal sums (48 used)
constexpr int kMxThreads = 256;
constexpr float kMxScale = 1024.f;

template <int C>
struct MxGeom {
  static constexpr int plane = kMxRows * kMxCols;                 // fp16 per channel plane
  static constexpr size_t planes = (size_t)C * plane * 2;
  static constexpr size_t keep = (size_t)kMxTX * kMxTY;
  static constexpr size_t hsum = (size_t)2 * 16 * kMxPT * 2;      // per wavefront: hi and lo parts
  static constexpr size_t taps = 64 * 4;                           // 2^10 x the taps, zero-padded
  static constexpr size_t lds = planes + keep + 4 * hsum + taps;
};

// in focus: depth inside one of the ranges
__device__ __forceinline__ bool in_focus(int dv, const BlurArgs& a) {
  bool k = false;
  for (int t = 0; t < a.nranges; ++t) k |= (dv >= a.lo[t] && dv <= a.hi[t]);
  return k;
}

// Two bytes b0, b1 as an fp16 pair: the perm puts each byte under an 0x64
// high byte (fp16 1024 + b), the packed subtraction removes the 1024 exactly.
__device__ __forceinline__ uint32_t byte_pair_f16(uint32_t word_with_64) {
  h16x2 v = __builtin_bit_cast(h16x2, word_with_64);
  v = v - (h16x2){(_Float16)1024.f, (_Float16)1024.f};
  return __builtin_bit_cast(uint32_t, v);
}

// The tiles: interior tiles (input columns x0 - 8 .. x0 + 71 inside the
// image) load their input as word groups; edge tiles byte by byte with
// clamped columns. Edge tiles take one workgroup each; interior
// tiles go to a persistent set of workgroups that load the next tile's
// words into registers while they sum and write the current one. Every lane
// of an interior tile issues the same loads and stores (rows clamped; the
// stores of pixels outside the image go to a sink word), so the wait for the
// next tile's loads never has to wait for the current tile's stores.
constexpr int kMxGroups = kMxCols / 4;                      // 4-pixel groups per input row
constexpr int kMxItems = kMxRows * kMxGroups;               // 960
constexpr int kMxPer = (kMxItems + kMxThreads - 1) / kMxThreads;
constexpr int kMxDWords = kMxTY * (kMxTX / 4) / kMxThreads; // depth words per thread: 2

struct MxTiles {
  int32_t ntx, nty;         // tiles per row and column
  int32_t ilo, icols;       // interior tile columns ilo .. ilo + icols - 1 (icols 0: none)
  int32_t ecols, nedge;     // edge tile columns per row; edge tiles
  int32_t ninner;           // interior tiles
  __device__ __forceinline__ int edge_cx(int ec) const { return icols == 0 ? ec : (ec == 0 ? 0 : ilo + icols - 1 + ec); }
};

// Words of a 4-pixel group as loaded: from the group's first byte when image
// rows are 4-byte aligned (3 words of RGB, 1 of grey), else from the word
// boundary below it (one word more, shifted into place when staged).
template <int C, bool kARows>
constexpr int kMxGroupWords = (C == 3 ? 3 : 1) + (kARows ? 0 : 1);

template <int C, bool kDWords, bool kARows>
struct MxLoads {
  uint32_t gw[kMxPer][kMxGroupWords<C, kARows>];
  uint32_t dv[kMxDWords][kDWords ? 1 : 2];   // depth words (from the word boundary below where rows are unaligned)
};

// first byte of 4-pixel group q of input row r (row clamped)
template <int C>
__device__ __forceinline__ const uint8_t* mx_group(const uint8_t* img, int H, int64_t pitch, int x0, int y0, int r,
                                                   int q) {
  const int yy = min(max(y0 - kMxRad + r, 0), H - 1);
  return img + (int64_t)yy * pitch + (int64_t)(x0 - kMxRad + 4 * q) * C;
}

// one interior tile's loads, the same for every lane and tile
template <int C, bool kDWords, bool kARows>
__device__ __forceinline__ void mx_issue(const uint8_t* img, const uint8_t* depth, int W, int H, int64_t pitch, int x0,
                                         int y0, int tid, MxLoads<C, kDWords, kARows>& L) {
#pragma unroll
  for (int k = 0; k < kMxPer; ++k) {
    const int ic = min(tid + k * kMxThreads, kMxItems - 1);   // past the last group: the last group again
    const int r = ic / kMxGroups, q = ic - r * kMxGroups;
    const uint8_t* src = mx_group<C>(img, H, pitch, x0, y0, r, q);
    if constexpr (!kARows) src = (const uint8_t*)((uintptr_t)src & ~(uintptr_t)3);
    constexpr int nw = kMxGroupWords<C, kARows>;
    if constexpr (nw == 4) {
      const u32x4 v = *(g_u32x4*)src;
      L.gw[k][0] = v.x; L.gw[k][1] = v.y; L.gw[k][2] = v.z; L.gw[k][3] = v.w;
    } else if constexpr (nw == 3) {
      const mu32x3 v = *(g_mu32x3*)src;
      L.gw[k][0] = v.x; L.gw[k][1] = v.y; L.gw[k][2] = v.z;
    } else if constexpr (nw == 2) {
      const mu32x2 v = *(g_mu32x2*)src;
      L.gw[k][0] = v.x; L.gw[k][1] = v.y;
    } else {
      L.gw[k][0] = *(g_mu32*)src;
    }
  }
#pragma unroll
  for (int k = 0; k < kMxDWords; ++k) {
    const int i = tid + k * kMxThreads;
    const int r = i / (kMxTX / 4), q = i - r * (kMxTX / 4);
    const uint8_t* d = depth + (int64_t)min(y0 + r, H - 1) * W + x0 + 4 * q;
    if constexpr (kDWords) {
      L.dv[k][0] = *(g_mu32*)d;
    } else {
      const mu32x2 v = *(g_mu32x2*)((uintptr_t)d & ~(uintptr_t)3);
      L.dv[k][0] = v.x; L.dv[k][1] = v.y;
    }
  }
}

// in-focus flags from an interior tile's depth loads (1 below the image);
// returns whether this thread saw a pixel to blur
template <bool kDWords>
__device__ __forceinline__ bool mx_flags_loaded(const uint32_t (*dv)[kDWords ? 1 : 2], const uint8_t* depth, int W,
                                                int H, int x0, int y0, int tid, uint8_t* keep, const BlurArgs& a) {
  bool need = false;
  const bool one = a.nranges == 1;
  const uint32_t lo = (uint32_t)a.lo[0], span = (uint32_t)(a.hi[0] - a.lo[0]);
  auto bit = [&](uint32_t d) -> uint32_t {
    return (one ? d - lo <= span : in_focus((int)d, a)) ? 1u : 0u;
  };
#pragma unroll
  for (int k = 0; k < kMxDWords; ++k) {
    const int i = tid + k * kMxThreads;
    const int r = i / (kMxTX / 4), q = i - r * (kMxTX / 4);
    uint32_t w = dv[k][0];
    if constexpr (!kDWords) {
      const uint32_t sh = (uint32_t)(uintptr_t)(depth + (int64_t)min(y0 + r, H - 1) * W + x0 + 4 * q) & 3u;
      w = __builtin_amdgcn_alignbyte(dv[k][1], dv[k][0], sh);
    }
    uint32_t kw = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) kw |= bit((w >> (8 * j)) & 0xFFu) << (8 * j);
    if (y0 + r >= H) kw = 0x01010101u;
    *(uint32_t*)(keep + r * kMxTX + 4 * q) = kw;
    need |= kw != 0x01010101u;
  }
  return need;
}

// in-focus flags read byte by byte (edge tiles)
__device__ __forceinline__ bool mx_flags_bytes(const uint8_t* depth, int W, int H, int x0, int y0, int tid,
                                               uint8_t* keep, const BlurArgs& a) {
  bool need = false;
  for (int i = tid; i < kMxTY * kMxTX; i += kMxThreads) {
    const int y = i / kMxTX, x = i - y * kMxTX;
    bool k = true;
    if (y0 + y < H && x0 + x < W) k = in_focus(depth[(int64_t)(y0 + y) * W + x0 + x], a);
    keep[i] = k ? 1 : 0;
    need |= !k;
  }
  return need;
}

// planar fp16 input tile from an interior tile's loaded groups
template <int C, bool kDWords, bool kARows>
__device__ __forceinline__ void mx_stage_loaded(const MxLoads<C, kDWords, kARows>& L, const uint8_t* img, int H,
                                                int64_t pitch, int x0, int y0, int tid, _Float16* P) {
  const uint32_t k64 = 0x64646464u;
#pragma unroll
  for (int k = 0; k < kMxPer; ++k) {
    const int i = tid + k * kMxThreads;
    if (i < kMxItems) {   // (the last wavefront's fourth group only)
      const int r = i / kMxGroups, q = i - r * kMxGroups;
      _Float16* dst = P + r * kMxCols + 4 * q;
      // the group's words, shifted into place when loaded from the word below
      uint32_t gw[C == 3 ? 3 : 1];
      if constexpr (kARows) {
#pragma unroll
        for (int j = 0; j < (C == 3 ? 3 : 1); ++j) gw[j] = L.gw[k][j];
      } else {
        const uint32_t sh = (uint32_t)(uintptr_t)mx_group<C>(img, H, pitch, x0, y0, r, q) & 3u;
#pragma unroll
        for (int j = 0; j < (C == 3 ? 3 : 1); ++j) gw[j] = __builtin_amdgcn_alignbyte(L.gw[k][j + 1], L.gw[k][j], sh);
      }
      if constexpr (C == 3) {
        const uint32_t w0 = gw[0], w1 = gw[1], w2 = gw[2];
        // w0 = R0 G0 B0 R1, w1 = G1 B1 R2 G2, w2 = B2 R3 G3 B3 (lowest byte first)
        const uint32_t r01 = byte_pair_f16(__builtin_amdgcn_perm(w0, k64, 0x00070004u));
        const uint32_t r23 = byte_pair_f16(__builtin_amdgcn_perm(w2, w1, 0x0c050c02u) | 0x64006400u);
        const uint32_t g01 = byte_pair_f16(__builtin_amdgcn_perm(w1, w0, 0x0c040c01u) | 0x64006400u);
        const uint32_t g23 = byte_pair_f16(__builtin_amdgcn_perm(w2, w1, 0x0c060c03u) | 0x64006400u);
        const uint32_t b01 = byte_pair_f16(__builtin_amdgcn_perm(w1, w0, 0x0c050c02u) | 0x64006400u);
        const uint32_t b23 = byte_pair_f16(__builtin_amdgcn_perm(w2, k64, 0x00070004u));
        constexpr int plane = MxGeom<C>::plane;
        *(mu32x2*)dst = (mu32x2){r01, r23};
        *(mu32x2*)(dst + plane) = (mu32x2){g01, g23};
        *(mu32x2*)(dst + 2 * plane) = (mu32x2){b01, b23};
      } else {
        const uint32_t w = gw[0];
        *(mu32x2*)dst = (mu32x2){byte_pair_f16(__builtin_amdgcn_perm(w, k64, 0x00050004u)),
                                 byte_pair_f16(__builtin_amdgcn_perm(w, k64, 0x00070006u))};
      }
    }
  }
}

// planar fp16 input tile byte by byte with clamped rows and columns (edge tiles)
template <int C>
__device__ __forceinline__ void mx_stage_bytes(const uint8_t* img, int W, int H, int64_t pitch, int x0, int y0, int tid,
                                               _Float16* P) {
  for (int e = tid; e < kMxRows * kMxCols * C; e += kMxThreads) {
    const int r = e / (kMxCols * C), jc = e - r * (kMxCols * C), j = jc / C, c = jc - j * C;
    const int yy = min(max(y0 - kMxRad + r, 0), H - 1), xx = min(max(x0 - kMxRad + j, 0), W - 1);
    P[c * MxGeom<C>::plane + r * kMxCols + j] = (_Float16)img[(int64_t)yy * pitch + (int64_t)xx * C + c];
  }
}

// The banded tap matrix, as this lane's eight entries (column n, rows
// 8g .. 8g + 7): taps[24 + t] holds 2^10 x tap t (zero outside [0, 2 radius]),
// a lane reads t = 8g + e - n - 8 + radius, in [-22, 31].
__device__ __forceinline__ void mx_weights(const float* taps, int rad, int n, int g, h16x8& whi, h16x8& wlo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float w = taps[24 + 8 * g + e - n - kMxRad + rad];
    const _Float16 hi = (_Float16)w;
    whi[e] = hi;
    wlo[e] = (_Float16)(w - (float)hi);
  }
}

// Both passes of one staged tile and its outputs (after the barrier that
// follows the staging). kSink: lanes outside the image store to `sink`.
template <int C, bool kSink>
__device__ __forceinline__ void mx_sum_store(const unsigned char* lds, int tid, bool need, const h16x8& whi,
                                             const h16x8& wlo, int x0, int y0, int W, int H, float* out, float* sink) {
  using G = MxGeom<C>;
  const _Float16* P = (const _Float16*)lds;
  const uint8_t* keep = lds + G::planes;
  const int wv = tid >> 6, l = tid & 63, n = l & 15, g = l >> 4;
  // this lane's outputs: rows 16p + 4g + i (p < 2, i < 4) of column 16 wv + n
  const int xx = 16 * wv + n;
  f32x4 res[C][2];
  if (need) {
    _Float16* hs = (_Float16*)(lds + G::planes + G::keep + (size_t)wv * G::hsum);   // [16][kMxPT] hi
    _Float16* hl = hs + 16 * kMxPT;                                                 // [16][kMxPT] lo
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const _Float16* pl = P + c * G::plane;
#pragma unroll
      for (int m = 0; m < kMxRows / 16; ++m) {
        // rows 16m .. 16m + 15 of the input tile, columns 16 wv .. 16 wv + 31
        const h16x8 A = *(const h16x8*)(pl + (16 * m + n) * kMxCols + 16 * wv + 8 * g);
        const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
        const f32x4 big = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, whi, zero, 0, 0, 0);
        const f32x4 small = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, wlo, zero, 0, 0, 0);
        // 2^10 x the horizontal sum of input row 16m + 4g + i at output column
        // 16 wv + n (the low taps' products summed apart: their roundings stay small)
        float h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = (big[i] + small[i]) * (1.f / kMxScale);
        const fp16x2 p0 = __builtin_amdgcn_cvt_pkrtz(h[0], h[1]);
        const fp16x2 p1 = __builtin_amdgcn_cvt_pkrtz(h[2], h[3]);
        const fp16x2 q0 = __builtin_amdgcn_cvt_pkrtz(h[0] - (float)p0.x, h[1] - (float)p0.y);
        const fp16x2 q1 = __builtin_amdgcn_cvt_pkrtz(h[2] - (float)p1.x, h[3] - (float)p1.y);
        *(mu32x2*)(hs + n * kMxPT + 16 * m + 4 * g) =
            (mu32x2){__builtin_bit_cast(uint32_t, p0), __builtin_bit_cast(uint32_t, p1)};
        *(mu32x2*)(hl + n * kMxPT + 16 * m + 4 * g) =
            (mu32x2){__builtin_bit_cast(uint32_t, q0), __builtin_bit_cast(uint32_t, q1)};
      }
      asm volatile("" ::: "memory");
#pragma unroll
      for (int p = 0; p < kMxTY / 16; ++p) {
        // horizontal sums of rows 16p .. 16p + 31 at this lane's column
        const h16x8 Bh = *(const h16x8*)(hs + n * kMxPT + 16 * p + 8 * g);
        const h16x8 Bl = *(const h16x8*)(hl + n * kMxPT + 16 * p + 8 * g);
        const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
        const f32x4 big = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, Bh, zero, 0, 0, 0);
        f32x4 small = __builtin_amdgcn_mfma_f32_16x16x32_f16(wlo, Bh, zero, 0, 0, 0);
        small = __builtin_amdgcn_mfma_f32_16x16x32_f16(whi, Bl, small, 0, 0, 0);
        res[c][p] = (big + small) * (1.f / kMxScale);   // the output at row 16p + 4g + i, column 16 wv + n
      }
      asm volatile("" ::: "memory");   // this channel's reads before the next channel's writes
    }
  } else {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int p = 0; p < 2; ++p) res[c][p] = (f32x4){0.f, 0.f, 0.f, 0.f};
  }

  // in-focus flags and input values of the lane's outputs, read at once
  uint32_t kf[2][4];
  float iv[C][2][4];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int yy = 16 * p + 4 * g + i;
      kf[p][i] = keep[yy * kMxTX + xx];
#pragma unroll
      for (int c = 0; c < C; ++c) iv[c][p][i] = (float)P[c * G::plane + (yy + kMxRad) * kMxCols + xx + kMxRad];
    }
  // outputs: in-focus pixels keep their input value
  float* o = out + ((int64_t)(y0 + 4 * g) * W + x0 + xx) * C;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int yy = 16 * p + 4 * g + i;
      const bool inside = y0 + yy < H && x0 + xx < W;
      if (!kSink && !inside) continue;
      float v[C];
#pragma unroll
      for (int c = 0; c < C; ++c) v[c] = kf[p][i] ? iv[c][p][i] : res[c][p][i];
      float* op = inside ? o + (int64_t)(16 * p + i) * W * C : sink;
      if constexpr (C == 3) {
        *(g_mu32x3_rw*)op = (mu32x3){__builtin_bit_cast(uint32_t, v[0]), __builtin_bit_cast(uint32_t, v[1]),
                                     __builtin_bit_cast(uint32_t, v[2])};
      } else {
        *(__attribute__((address_space(1))) float*)op = v[0];
      }
    }
}

// flags bit 0: image rows start on 4-byte boundaries. Workgroups below
// T.nedge take one edge tile each; the others walk the interior tiles.
template <int C, bool kDWords, bool kARows>
__global__ __launch_bounds__(kMxThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_blur_mfma(
    const uint8_t* img, const uint8_t* depth, int32_t W, int32_t H, int64_t pitch, BlurArgs a, float* out, float* sink,
    MxTiles T) {
  using G = MxGeom<C>;
  extern __shared__ __attribute__((aligned(16))) unsigned char mx_lds[];
  _Float16* P = (_Float16*)mx_lds;
  uint8_t* keep = mx_lds + G::planes;
  float* taps = (float*)(mx_lds + G::planes + G::keep + 4 * G::hsum);
  const int tid = threadIdx.x;
  const int n = tid & 15, g = (tid & 63) >> 4;
  if (tid < 64) {
    const int t = tid - 24;
    taps[tid] = (t >= 0 && t <= 2 * a.rad) ? a.g[t] * kMxScale : 0.f;
  }

  if ((int)blockIdx.x < T.nedge) {
    const int e = blockIdx.x;
    const int x0 = T.edge_cx(e % T.ecols) * kMxTX, y0 = (e / T.ecols) * kMxTY;
    bool need = mx_flags_bytes(depth, W, H, x0, y0, tid, keep, a);
    mx_stage_bytes<C>(img, W, H, pitch, x0, y0, tid, P);
    need = __syncthreads_or(need);
    h16x8 whi, wlo;
    mx_weights(taps, a.rad, n, g, whi, wlo);
    mx_sum_store<C, false>(mx_lds, tid, need, whi, wlo, x0, y0, W, H, out, sink);
    return;
  }
  // interior tiles
  const int step = gridDim.x - T.nedge;
  int t = blockIdx.x - T.nedge;
  if (t >= T.ninner) return;
  auto origin = [&](int tt, int& x0, int& y0) {
    x0 = (T.ilo + tt % T.icols) * kMxTX;
    y0 = (tt / T.icols) * kMxTY;
  };
  MxLoads<C, kDWords, kARows> L;
  {
    int x0, y0;
    origin(t, x0, y0);
    mx_issue<C, kDWords, kARows>(img, depth, W, H, pitch, x0, y0, tid, L);
  }
  h16x8 whi, wlo;
  bool have_w = false;
  for (; t < T.ninner; t += step) {
    int x0, y0;
    origin(t, x0, y0);
    __syncthreads();   // the previous tile's reads of the LDS are done (and the taps are written)
    if (!have_w) { mx_weights(taps, a.rad, n, g, whi, wlo); have_w = true; }
    bool need = mx_flags_loaded<kDWords>(L.dv, depth, W, H, x0, y0, tid, keep, a);
    mx_stage_loaded<C, kDWords, kARows>(L, img, H, pitch, x0, y0, tid, P);
    if (t + step < T.ninner) {
      int nx0, ny0;
      origin(t + step, nx0, ny0);
      mx_issue<C, kDWords, kARows>(img, depth, W, H, pitch, nx0, ny0, tid, L);   // in flight while this tile is finished
    }
    need = __syncthreads_or(need);
    mx_sum_store<C, true>(mx_lds, tid, need, whi, wlo, x0, y0, W, H, out, sink);
  }
}

template <int C>
void launch_blur_mfma(hipStream_t s, const uint8_t* img, const uint8_t* depth, int32_t W, int32_t H, int64_t pitch,
                      bool img_words, bool depth_words, const BlurArgs& a, float* out, float* sink) {
  MxTiles T{};
  T.ntx = (W + kMxTX - 1) / kMxTX;
  T.nty = (H + kMxTY - 1) / kMxTY;
  // interior columns: cx >= 1 and 64 cx + 72 <= W (+ 4 where image rows are
  // not word-aligned: a group's words are loaded from the word boundary below
  // it, up to 4 bytes past the tile's last input byte)
  const int reach = kMxTX + kMxRad + (img_words ? 0 : 4);
  const int ihi = W >= reach ? (W - reach) / kMxTX : 0;
  T.ilo = 1;
  T.icols = ihi >= 1 ? ihi : 0;
  T.ecols = T.ntx - T.icols;
  T.nedge = T.ecols * T.nty;
  T.ninner = T.icols * T.nty;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // four workgroups fit a CU's LDS
  const int inner_groups = std::min(T.ninner, 4 * std::max(cus, 1));
  const dim3 grid((unsigned)(T.nedge + inner_groups));
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(kMxThreads), MxGeom<C>::lds, s, img, depth, W, H, pitch, a, out, sink, T);
  };
  if (img_words) {
    if (depth_words) go(k_blur_mfma<C, true, true>);
    else go(k_blur_mfma<C, false, true>);
  } else {
    if (depth_words) go(k_blur_mfma<C, true, false>);
    else go(k_blur_mfma<C, false, false>);
  }
}

int fail(int st, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return sbs::report_error(st, buf);
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace sbs_post

using namespace sbs_post;

extern "C" {

size_t sbs_reconstruct_workspace_bytes(int32_t W, int32_t H) {
  if (W < 1 || H < 1) return 0;
  const size_t N = (size_t)W * H;
  return align256(N * 4) + align256(N * 2) + align256(N * 2);
}

int sbs_reconstruct(const uint32_t* idx, const uint8_t* disp, int64_t n, int32_t W, int32_t H, int32_t threshold,
                    uint8_t* out_map, void* workspace, size_t workspace_bytes, void* stream) {
  if (W < 1 || H < 1 || (int64_t)W * H > INT32_MAX) return fail(SBS_ERR_INVALID_ARG, "bad W/H");
  if (n < 0 || n > INT32_MAX) return fail(SBS_ERR_INVALID_ARG, "bad n");
  if (!out_map || !workspace || (n > 0 && (!idx || !disp))) return fail(SBS_ERR_INVALID_ARG, "NULL pointer");
  if (threshold < 0) return fail(SBS_ERR_INVALID_ARG, "threshold < 0");
  if (workspace_bytes < sbs_reconstruct_workspace_bytes(W, H)) return fail(SBS_ERR_INVALID_ARG, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = (int64_t)W * H;
  char* base = (char*)workspace;
  int32_t* slot = (int32_t*)base;
  int16_t* f = (int16_t*)(base + align256(N * 4));
  int16_t* up = (int16_t*)(base + align256(N * 4) + align256(N * 2));
  hipLaunchKernelGGL(k_rc_clear, dim3(1024), dim3(256), 0, s, slot, N);
  if (n > 0) {
    const unsigned sg = (unsigned)std::min<int64_t>((n + 1023) / 1024, 2048);
    hipLaunchKernelGGL(k_rc_scatter, dim3(sg), dim3(256), 0, s, idx, n, N, slot);
    hipLaunchKernelGGL(k_rc_scatter_max, dim3(sg), dim3(256), 0, s, idx, n, N, slot);
  }
  hipLaunchKernelGGL(k_rc_fill, dim3(H < 65536 ? H : 65536), dim3(kRowThreads), 0, s, slot, disp, W, H, f);
  // The column pass's segment records and their chunk summaries reuse the
  // slot array (no longer read after k_rc_fill): 2 x (nseg + nch) x W int16,
  // within its 4 x W x H bytes (summaries only when nch > 1, i.e. H > 256:
  // then nseg + nch <= H / 16 + H / 256 + 2 < H).
  const int seglen = std::max(kColSeg, (H + 65534) / 65535);
  const int nseg = (H + seglen - 1) / seglen;
  int16_t* seg_first = (int16_t*)slot;
  int16_t* seg_last = seg_first + (int64_t)nseg * W;
  const dim3 cg((W + 255) / 256, nseg);
  hipLaunchKernelGGL(k_rc_colseg, cg, dim3(256), 0, s, f, W, H, seglen, seg_first, seg_last);
  // chunk summaries after the segment records, still inside the slot array
  const int nch = (nseg + kScanBatch - 1) / kScanBatch;
  int16_t* ch_first = seg_last + (int64_t)nseg * W;
  int16_t* ch_last = ch_first + (int64_t)nch * W;
  const dim3 chg((W + 255) / 256, nch);
  // (one chunk: no carries to take, and no room needed for summaries)
  if (nch > 1) {
    hipLaunchKernelGGL(k_rc_chunks, chg, dim3(256), 0, s, W, nseg, seg_first, seg_last, ch_first, ch_last);
    hipLaunchKernelGGL(k_rc_colscan, dim3((W + 255) / 256), dim3(256), 0, s, W, nch, ch_first, ch_last);
  }
  hipLaunchKernelGGL(k_rc_segscan, chg, dim3(256), 0, s, W, nseg, seg_first, seg_last, ch_first, ch_last);
  hipLaunchKernelGGL(k_rc_peek, cg, dim3(256), 0, s, f, W, H, threshold, seglen, seg_last, seg_first, up, out_map);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SBS_ERR_HIP, "reconstruct: %s", hipGetErrorString(e));
  return SBS_OK;
}

size_t sbs_selective_blur_workspace_bytes(int32_t W, int32_t H, int32_t C) {
  if (W < 1 || H < 1 || (C != 1 && C != 3)) return 0;
  return align256((size_t)W * H * C * 4);
}

int sbs_selective_blur(const uint8_t* img, int32_t W, int32_t H, int32_t C, int64_t pitch, const uint8_t* depth,
                       const int32_t* ranges, int32_t nranges, float sigma, float* out, void* workspace,
                       size_t workspace_bytes, void* stream) {
  if (W < 1 || H < 1 || (C != 1 && C != 3) || pitch < (int64_t)W * C) return fail(SBS_ERR_INVALID_ARG, "bad image");
  if (!img || !depth || !out || !workspace) return fail(SBS_ERR_INVALID_ARG, "NULL pointer");
  if (nranges < 0 || nranges > kMaxRanges || (nranges > 0 && !ranges))
    return fail(SBS_ERR_INVALID_ARG, "nranges must be in [0, %d]", kMaxRanges);
  if (!(sigma > 0.f)) return fail(SBS_ERR_INVALID_ARG, "sigma must be > 0");
  const int rad = (int)std::ceil(3.0 * (double)sigma);
  if (rad > kMaxRadius) return fail(SBS_ERR_UNSUPPORTED, "sigma too large (radius %d > %d)", rad, kMaxRadius);
  if (workspace_bytes < sbs_selective_blur_workspace_bytes(W, H, C)) return fail(SBS_ERR_INVALID_ARG, "workspace too small");
  if (((uintptr_t)workspace & 3) != 0) return fail(SBS_ERR_INVALID_ARG, "workspace not 4-byte aligned");
  BlurArgs a{};
  double gs = 0.0;
  double g[2 * kMaxRadius + 1];
  for (int k = -rad; k <= rad; ++k) { g[k + rad] = std::exp(-(double)(k * k) / (2.0 * (double)sigma * sigma)); gs += g[k + rad]; }
  for (int k = 0; k <= 2 * rad; ++k) a.g[k] = (float)(g[k] / gs);
  a.rad = rad;
  a.nranges = nranges;
  for (int t = 0; t < nranges; ++t) { a.lo[t] = ranges[2 * t]; a.hi[t] = ranges[2 * t + 1]; }
  hipStream_t s = (hipStream_t)stream;
  const int64_t mx_tiles = (int64_t)((W + kMxTX - 1) / kMxTX) * ((H + kMxTY - 1) / kMxTY);
  if (rad <= kMxRad && mx_tiles < (1LL << 30)) {
    const bool img_words = (((uintptr_t)img | (uintptr_t)pitch) & 3) == 0;
    const bool depth_words = (((uintptr_t)depth | (uintptr_t)W) & 3) == 0;
    float* sink = (float*)workspace;   // stores of lanes outside the image (12 bytes)
    if (C == 3) launch_blur_mfma<3>(s, img, depth, W, H, pitch, img_words, depth_words, a, out, sink);
    else launch_blur_mfma<1>(s, img, depth, W, H, pitch, img_words, depth_words, a, out, sink);
  } else if (rad <= kBlurTileRad && (H + kBlurTY - 1) / kBlurTY <= 65535) {
    const int64_t tx = (W + kBlurTX - 1) / kBlurTX;
    const dim3 grid((unsigned)tx, (unsigned)((H + kBlurTY - 1) / kBlurTY));
    const int32_t aligned = (((uintptr_t)img | (uintptr_t)pitch) & 3) == 0 ? 1 : 0;
    const auto radii = std::make_integer_sequence<int, kBlurTileRad>{};
    if (C == 3) blur_tile_dispatch<3>(rad, radii, grid, s, img, depth, W, H, pitch, aligned, a, out);
    else blur_tile_dispatch<1>(rad, radii, grid, s, img, depth, W, H, pitch, aligned, a, out);
  } else {
    float* tmp = (float*)workspace;
    hipLaunchKernelGGL(k_blur_h, dim3(2048), dim3(256), 0, s, img, W, H, C, pitch, a, tmp);
    hipLaunchKernelGGL(k_blur_v, dim3(2048), dim3(256), 0, s, img, depth, W, H, C, pitch, a, tmp, out);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SBS_ERR_HIP, "blur: %s", hipGetErrorString(e));
  return SBS_OK;
}

}  // extern "C"
