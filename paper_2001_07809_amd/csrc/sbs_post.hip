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

__global__ __launch_bounds__(256) void k_rc_scatter(const uint32_t* idx, int64_t n, int64_t N, int32_t* slot) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = idx[k];
    if ((int64_t)p < N) atomicMax(&slot[p], (int32_t)k);
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
// bottommost determined value, k_rc_segscan turns those records into the
// nearest determined value above and below each segment (one pass down and
// one up each column, so a column with few determined pixels costs O(nseg),
// not O(nseg^2)), and k_rc_peek resolves the segment's rows in two passes
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
  for (int y = y0; y < y1; ++y) {
    const int16_t v = f[(int64_t)y * W + x];
    if (v >= 0) {
      if (first < 0) first = v;
      last = v;
    }
  }
  seg_first[(int64_t)sg * W + x] = first;
  seg_last[(int64_t)sg * W + x] = last;
}

// In place: seg_last[sg] becomes the nearest determined value above segment
// sg (the last one of the segments before it), seg_first[sg] the nearest
// below it (the first one of the segments after it); -1 where none. The
// records are read kScanBatch at a time before any of them is written, so a
// thread has that many loads in flight instead of one round trip per segment.
constexpr int kScanBatch = 16;
__global__ __launch_bounds__(256) void k_rc_segscan(int32_t W, int32_t nseg, int16_t* seg_first, int16_t* seg_last) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= W) return;
  int16_t carry = -1;
  for (int s0 = 0; s0 < nseg; s0 += kScanBatch) {
    int16_t v[kScanBatch];
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) v[k] = s0 + k < nseg ? seg_last[(int64_t)(s0 + k) * W + x] : (int16_t)-1;
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) {
      if (s0 + k >= nseg) break;
      seg_last[(int64_t)(s0 + k) * W + x] = carry;
      if (v[k] >= 0) carry = v[k];
    }
  }
  carry = -1;
  for (int s1 = nseg - 1; s1 >= 0; s1 -= kScanBatch) {   // segments s1, s1 - 1, ...
    int16_t v[kScanBatch];
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) v[k] = s1 - k >= 0 ? seg_first[(int64_t)(s1 - k) * W + x] : (int16_t)-1;
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) {
      if (s1 - k < 0) break;
      seg_first[(int64_t)(s1 - k) * W + x] = carry;
      if (v[k] >= 0) carry = v[k];
    }
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
  if (n > 0) hipLaunchKernelGGL(k_rc_scatter, dim3(256), dim3(256), 0, s, idx, n, N, slot);
  hipLaunchKernelGGL(k_rc_fill, dim3(H < 65536 ? H : 65536), dim3(kRowThreads), 0, s, slot, disp, W, H, f);
  // The column pass's segment records reuse the slot array (no longer read
  // after k_rc_fill): 2 x nseg x W int16 <= 4 x W x H bytes.
  const int seglen = std::max(kColSeg, (H + 65534) / 65535);
  const int nseg = (H + seglen - 1) / seglen;
  int16_t* seg_first = (int16_t*)slot;
  int16_t* seg_last = seg_first + (int64_t)nseg * W;
  const dim3 cg((W + 255) / 256, nseg);
  hipLaunchKernelGGL(k_rc_colseg, cg, dim3(256), 0, s, f, W, H, seglen, seg_first, seg_last);
  hipLaunchKernelGGL(k_rc_segscan, dim3((W + 255) / 256), dim3(256), 0, s, W, nseg, seg_first, seg_last);
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
  BlurArgs a{};
  double gs = 0.0;
  double g[2 * kMaxRadius + 1];
  for (int k = -rad; k <= rad; ++k) { g[k + rad] = std::exp(-(double)(k * k) / (2.0 * (double)sigma * sigma)); gs += g[k + rad]; }
  for (int k = 0; k <= 2 * rad; ++k) a.g[k] = (float)(g[k] / gs);
  a.rad = rad;
  a.nranges = nranges;
  for (int t = 0; t < nranges; ++t) { a.lo[t] = ranges[2 * t]; a.hi[t] = ranges[2 * t + 1]; }
  hipStream_t s = (hipStream_t)stream;
  if (rad <= kBlurTileRad) {
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
