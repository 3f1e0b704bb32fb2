// The step before the disparity search (arXiv 2001.07809, Sec. III): from a
// left image to the ascending list of its refined segment-boundary pixels.
//   lightness      CIE L* of each pixel, scaled to 8 bits ("Colour Space
//                  Conversion"); gray images pass through
//   histogram      256 bins of lightness ("Segmentation")
//   k-means        on the bins, distance |a - b|, exact rational centres
//   labels         each pixel takes its bin's cluster, renumbered by
//                  ascending centre
//   refinement     configured: 3x3 open then close on the labels; paper:
//                  Moore-neighbour boundary, then 'fill', then 'remove'
//                  ("Segment Boundary Detection", "Refinement")
//   components     8-connected components of the boundary map by lock-free
//                  union-find; each root is its component's smallest raster
//                  index
//   filter         configured: keep components of at least min_cc pixels;
//                  paper: drop the smallest components (ties by raster order)
//                  while the dropped total stays within 4% of all boundary
//                  pixels
//   list           left and right border columns plus the kept pixels, in
//                  ascending raster order ("Disparity Measurement": pixels on
//                  the left/right borders of the map count as boundary)
// Declared in include/sbs.h.
#include <hip/hip_runtime.h>
#include <cstring>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "../../include/sbs.h"
#include "sbs_internal.h"

namespace sbs_front {

constexpr int kBlock = 256;
constexpr int kScanPer = 1024;     // elements per block in the device-wide scans
constexpr int kRsPasses = 8;       // most counting passes of one radix select (a 64-bit key)
constexpr int kMaxK = 64;
constexpr int kMaxPasses = 1000;
constexpr int kN1Parts = 64;        // partial counts of kept pixels (fraction control)
constexpr int kMiscBytes = 2048;    // small device state of one call, cleared at its start

// ---------------------------------------------------------------------------
// Lightness. sRGB decode of each channel, luminance Y = 0.2126 R + 0.7152 G +
// 0.0722 B on linear values, L* = 116 f(Y) - 16 with f the CIE cube-root law
// (linear below (6/29)^3), scaled by 255/100 and rounded half away from zero.
// fp64 without contraction: every product and sum is rounded on its own.
__device__ __forceinline__ double srgb_linear(int v) {
#pragma clang fp contract(off)
  const double c = v / 255.0;
  return c <= 0.04045 ? c / 12.92 : pow((c + 0.055) / 1.055, 2.4);
}

// L8 as a function of Y is a non-decreasing step function, so a pixel's
// value is the number of steps at or below its Y: t[v] (v = 1 .. 255) is the
// smallest Y whose L8 is at least v (+inf if none). The table comes from the
// host (light_steps below); the kernel then needs no cube root per pixel.
struct LightSteps {
  double t[256];
};

__global__ __launch_bounds__(kBlock) void k_light(const uint8_t* __restrict__ img, int32_t W, int32_t H, int32_t C,
                                                  int64_t pitch, uint8_t* __restrict__ L8, LightSteps steps) {
#pragma clang fp contract(off)
  __shared__ double lin[256];
  __shared__ double t[256];
  if (C == 3) {
    lin[threadIdx.x] = srgb_linear((int)threadIdx.x);
    t[threadIdx.x] = steps.t[threadIdx.x];
    __syncthreads();
  }
  const int64_t N = (int64_t)W * H;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)((uint32_t)i / (uint32_t)W), x = (int)((uint32_t)i % (uint32_t)W);   // N < 2^31
    const uint8_t* p = img + (int64_t)y * pitch + (int64_t)x * C;
    if (C == 1) { L8[i] = p[0]; continue; }
    const double Y = 0.2126 * lin[p[0]] + 0.7152 * lin[p[1]] + 0.0722 * lin[p[2]];
    int v = 0;
#pragma unroll
    for (int st = 128; st; st >>= 1)
      if (Y >= t[v + st]) v += st;
    L8[i] = (uint8_t)v;
  }
}

// Gray images: L8 is the image itself (rows gathered from the pitch).
__global__ __launch_bounds__(kBlock) void k_gray(const uint8_t* __restrict__ img, int32_t W, int32_t H, int64_t pitch,
                                                 uint8_t* __restrict__ L8) {
  const int64_t N = (int64_t)W * H;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)((uint32_t)i / (uint32_t)W), x = (int)((uint32_t)i % (uint32_t)W);   // N < 2^31
    L8[i] = img[(int64_t)y * pitch + x];
  }
}

// RGB rows whose width is a multiple of 4 at word-aligned addresses: four
// pixels per thread from three aligned words, one word written.
// Four pixels per thread from three aligned words. The step search starts
// from a table over Y in 1/4096 buckets: coarse[b] is the last step at or
// below b/4096, and since consecutive steps lie more than 1/4096 apart (the
// host checks it before it takes this kernel) a bucket holds at most one
// step, so one comparison finishes the search (instead of eight dependent
// LDS reads). Built per block from the steps, for a grid of a few blocks per CU.
constexpr int kLightBuckets = 4096;
__global__ __launch_bounds__(kBlock) void k_light4(const uint8_t* __restrict__ img, int32_t W, int32_t H,
                                                   int64_t pitch, uint8_t* __restrict__ L8, LightSteps steps) {
#pragma clang fp contract(off)
  __shared__ double lin[256];
  __shared__ double t[256];
  __shared__ uint8_t coarse[kLightBuckets + 1];
  lin[threadIdx.x] = srgb_linear((int)threadIdx.x);
  t[threadIdx.x] = steps.t[threadIdx.x];
  __syncthreads();
  {
    // step k covers buckets ceil(t[k] 4096) .. ceil(t[k + 1] 4096) - 1 (step 0 from bucket 0)
    const int k = threadIdx.x;
    auto first_bucket = [&](int j) -> int {
      return j > 255 ? kLightBuckets + 1 : (int)fmin(ceil(t[j] * (double)kLightBuckets), (double)(kLightBuckets + 1));
    };
    const int b0 = k == 0 ? 0 : first_bucket(k), b1 = first_bucket(k + 1);
    for (int b = b0; b < b1; ++b) coarse[b] = (uint8_t)k;
  }
  __syncthreads();
  const int64_t Q = (int64_t)W * H / 4;   // groups of four pixels (W % 4 == 0)
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < Q; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = 4 * g;
    const int y = (int)((uint32_t)i / (uint32_t)W), x = (int)((uint32_t)i % (uint32_t)W);   // N < 2^31
    const uint32_t* p = (const uint32_t*)(img + (int64_t)y * pitch + (int64_t)x * 3);
    const uint32_t w0 = p[0], w1 = p[1], w2 = p[2];
    const uint32_t px[4][3] = {{w0 & 0xFFu, (w0 >> 8) & 0xFFu, (w0 >> 16) & 0xFFu},
                               {w0 >> 24, w1 & 0xFFu, (w1 >> 8) & 0xFFu},
                               {(w1 >> 16) & 0xFFu, w1 >> 24, w2 & 0xFFu},
                               {(w2 >> 8) & 0xFFu, (w2 >> 16) & 0xFFu, w2 >> 24}};
    uint32_t out = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double Y = 0.2126 * lin[px[k][0]] + 0.7152 * lin[px[k][1]] + 0.0722 * lin[px[k][2]];
      int v = coarse[min((int)(Y * (double)kLightBuckets), kLightBuckets)];   // Y >= 0
      if (v < 255 && Y >= t[v + 1]) ++v;
      out |= (uint32_t)v << (8 * k);
    }
    *(uint32_t*)(L8 + i) = out;
  }
}

// Lightness of an image on `s`: the four-pixel kernel where its layout allows.
void launch_light(const uint8_t* img, int32_t W, int32_t H, int32_t C, int64_t pitch, uint8_t* L8, int grid,
                  hipStream_t s);

__global__ __launch_bounds__(kBlock) void k_fill(uint8_t* p, int64_t n, uint8_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Histogram: 16-byte loads (16 pixels per thread and step where the buffer
// is 16-byte aligned), LDS atomic adds into 16 copies of the bins (lane l
// uses copy l % 16; copies are 257 words apart, so equal values in different
// copies fall in different banks), then one global add per bin and block.
constexpr int kHistCopies = 16;
__global__ __launch_bounds__(kBlock) void k_hist(const uint8_t* __restrict__ L8, int64_t N,
                                                 unsigned long long* __restrict__ hist) {
  __shared__ uint32_t h[kHistCopies][257];
  for (int i = threadIdx.x; i < kHistCopies * 257; i += blockDim.x) (&h[0][0])[i] = 0u;
  __syncthreads();
  uint32_t* mine = h[threadIdx.x & (kHistCopies - 1)];
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  int64_t head = 0;
  if (((uintptr_t)L8 & 15u) == 0) {
    const int64_t nv = N >> 4;
    for (int64_t v = tid; v < nv; v += stride) {
      const uint4 q = *(const uint4*)(L8 + 16 * v);
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int b = 0; b < 4; ++b) atomicAdd(&mine[(w[j] >> (8 * b)) & 0xFFu], 1u);
    }
    head = nv << 4;
  }
  for (int64_t i = head + tid; i < N; i += stride) atomicAdd(&mine[L8[i]], 1u);
  __syncthreads();
  uint32_t t = 0;
  for (int c = 0; c < kHistCopies; ++c) t += h[c][threadIdx.x];
  if (t) atomicAdd(&hist[threadIdx.x], (unsigned long long)t);
}

// K-means on the occupied bins, one block, thread b owns bin b. Centres are
// S_k / N_k (exact rationals); start c_k = Lmin + floor((2k+1)(Lmax-Lmin+1) /
// 2K) with N_k = 1; a bin goes to the nearest centre, ties to the lower k; an
// empty cluster keeps its centre; passes stop when no bin changes (at most
// 1000). Clusters are then renumbered by ascending centre (ties by index).
// Output: lut[b] = label of bin b (0 for empty bins).
__global__ __launch_bounds__(256) void k_kmeans(const unsigned long long* __restrict__ hist, int32_t K,
                                                uint8_t* __restrict__ lut, int32_t* __restrict__ passes_out) {
  __shared__ long long S[kMaxK], Nn[kMaxK];
  __shared__ double M[kMaxK];   // S / N rounded to double
  __shared__ unsigned long long s2[kMaxK], n2[kMaxK];
  __shared__ int lo_s, hi_s, changed;
  __shared__ int rank[kMaxK];
  const int b = threadIdx.x;
  const long long hb = (long long)hist[b];
  if (b == 0) { lo_s = 256; hi_s = -1; }
  __syncthreads();
  if (hb > 0) { atomicMin(&lo_s, b); atomicMax(&hi_s, b); }
  __syncthreads();
  const int lo = lo_s, hi = hi_s;
  if (hi < 0) {   // empty image cannot occur (N >= 1), kept for completeness
    lut[b] = 0;
    if (b == 0) *passes_out = 0;
    return;
  }
  if (b < K) { S[b] = lo + ((long long)(2 * b + 1) * (hi - lo + 1)) / (2 * K); Nn[b] = 1; }
  int assign = -1;
  int pass = 0;
  for (; pass < kMaxPasses; ++pass) {
    if (b == 0) changed = 0;
    if (b < K) {
      s2[b] = 0;
      n2[b] = 0;
      M[b] = (double)S[b] / (double)Nn[b];   // S < 2^40 and N < 2^32: both exact, the quotient rounded once
    }
    __syncthreads();
    if (hb > 0) {
      // |b - S_k/N_k| < |b - S_best/N_best|, decided on the rounded means
      // where they differ by more than their rounding (|error| < 2^-44 for
      // means in [0, 255]), else exactly:
      //   |b N_k - S_k| N_best < |b N_best - S_best| N_k
      int best = 0;
      long long Sb = S[0], Nb = Nn[0];
      double db = fabs((double)b - M[0]);
      for (int k = 1; k < K; ++k) {
        const double dk = fabs((double)b - M[k]);
        bool closer;
        if (dk < db - 0x1p-40) closer = true;
        else if (dk > db + 0x1p-40) closer = false;
        else {
          const long long Sk = S[k], Nk = Nn[k];
          closer = (__int128)llabs((long long)b * Nk - Sk) * Nb < (__int128)llabs((long long)b * Nb - Sb) * Nk;
        }
        if (closer) { best = k; db = dk; Sb = S[k]; Nb = Nn[k]; }
      }
      if (assign != best) { assign = best; changed = 1; }
    }
    __syncthreads();
    const int ch = changed;
    if (!ch && pass > 0) break;
    if (hb > 0) {
      atomicAdd(&s2[assign], (unsigned long long)(b * hb));
      atomicAdd(&n2[assign], (unsigned long long)hb);
    }
    __syncthreads();
    if (b < K && n2[b] > 0) { S[b] = (long long)s2[b]; Nn[b] = (long long)n2[b]; }
    __syncthreads();
    if (!ch) break;
  }
  if (b < K) {
    int rk = 0;
    for (int j = 0; j < K; ++j) {
      const __int128 a = (__int128)S[j] * Nn[b], c = (__int128)S[b] * Nn[j];
      rk += (a < c) || (a == c && j < b);
    }
    rank[b] = rk;
  }
  __syncthreads();
  lut[b] = assign < 0 ? 0 : (uint8_t)rank[assign];
  if (b == 0) *passes_out = pass + 1;
}

__global__ __launch_bounds__(kBlock) void k_label(const uint8_t* __restrict__ L8, int64_t N,
                                                  const uint8_t* __restrict__ lut, uint8_t* __restrict__ lab) {
  __shared__ uint8_t t[256];
  t[threadIdx.x] = lut[threadIdx.x];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    lab[i] = t[L8[i]];
}

// ---------------------------------------------------------------------------
// 3x3 refinement stencils (one fused kernel per mode below):
//   erosion (min) and dilation (max) with replicate borders;
//   Moore boundary: 1 iff an in-image 8-neighbour differs;
//   'fill': a 0 whose eight neighbours are all 1 becomes 1 (outside = 0);
//   'remove': a 1 whose four 4-neighbours are all 1 becomes 0 (outside = 0).

// The configured refinement in one pass over the image: erode, dilate
// (open), dilate, erode (close) with replicate borders, then the Moore
// boundary, per tile of kMorphT x kMorphT pixels with a 5-pixel halo held in
// LDS (one HBM read of the labels and one write of the boundary map, instead
// of five of each). Each step runs on a box one pixel narrower on every side
// than the one before, so its neighbours are always in the box. Clamping a
// neighbour into the image is the same as reading a frame whose cells
// outside the image repeat the nearest cell inside: the labels are loaded
// that way, and on tiles at an image edge every step's result is repeated
// into its outside cells before the next step reads them. The boundary step
// ignores neighbours outside the image. `closed`
// (optional) receives the labels after the close.
constexpr int kMorphT = 64, kMorphHalo = 5, kMorphF = kMorphT + 2 * kMorphHalo;   // frame: 74 x 74
constexpr int kMorphP = 84;   // LDS row pitch: a multiple of 4 with room for the word-wide reads past the frame

// Per-byte minimum / maximum of four labels packed in a word (labels < 128:
// (a | 0x80) - b keeps each byte apart, and its bit 7 says a >= b).
__device__ __forceinline__ uint32_t ge_mask4(uint32_t a, uint32_t b) {
  return ((((a | 0x80808080u) - b) >> 7) & 0x01010101u) * 0xFFu;
}
__device__ __forceinline__ uint32_t min4(uint32_t a, uint32_t b) { const uint32_t m = ge_mask4(a, b); return (b & m) | (a & ~m); }
__device__ __forceinline__ uint32_t max4(uint32_t a, uint32_t b) { const uint32_t m = ge_mask4(a, b); return (a & m) | (b & ~m); }

// Four cells per thread and step, from two aligned LDS words per row and
// byte shifts. A step on the box inset by k reads its source from column
// fx - 1; the buffer it writes keeps frame column c at byte c + (-k mod 4),
// so that the next step's reads start on a word again (the loaded frame has
// offset 0, and so has the closed frame the boundary step reads). Groups at
// a box's right end spill up to three cells past it; no later step reads
// those. Frames inside the image with rows of whole words load and store
// words; the others load bytes with clamped coordinates and store bytes,
// and at an image edge every step's cells outside the image are then set to
// the nearest cell inside, and the boundary of cells on the image's border
// rows and columns is taken again without the neighbours outside.
__global__ __launch_bounds__(kBlock) void k_morph_refine(const uint8_t* __restrict__ lab, int32_t W, int32_t H,
                                                         uint8_t* __restrict__ B, uint8_t* __restrict__ closed,
                                                         int32_t words) {
  __shared__ __attribute__((aligned(16))) uint8_t buf[2][kMorphF * kMorphP];
  const int x0 = blockIdx.x * kMorphT - kMorphHalo, y0 = blockIdx.y * kMorphT - kMorphHalo;   // frame origin
  const bool edge = x0 < 0 || y0 < 0 || x0 + kMorphF > W || y0 + kMorphF > H;
  const bool wide = !edge && words;   // word loads and stores
  if (wide) {
    constexpr int kWords = (kMorphF + 3 + 3) / 4;   // global words covering a frame row from column x0 - 3
    for (int c = threadIdx.x; c < kMorphF * kWords; c += kBlock) {
      const int fy = c / kWords, w = c - fy * kWords;
      const uint8_t* row = lab + (int64_t)(y0 + fy) * W;
      const int g0 = x0 - 3 + 4 * w;   // a multiple of 4 (x0 = 64 bx - 5)
      uint32_t v = 0u;
      if (g0 + 3 < W) v = *(const uint32_t*)(row + g0);
      else
        for (int j = 0; j < 4; ++j)
          if (g0 + j < W) v |= (uint32_t)row[g0 + j] << (8 * j);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int fx = 4 * w + j - 3;
        if (fx >= 0 && fx < kMorphF) buf[0][fy * kMorphP + fx] = (uint8_t)(v >> (8 * j));
      }
    }
  } else {
    constexpr int kPer = (kMorphF * kMorphF + kBlock - 1) / kBlock;
    uint8_t v[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int c = threadIdx.x + i * kBlock;
      v[i] = 0;
      if (c < kMorphF * kMorphF) {
        const int fy = c / kMorphF, fx = c - fy * kMorphF;
        const int gy = min(max(y0 + fy, 0), H - 1), gx = min(max(x0 + fx, 0), W - 1);
        v[i] = lab[(int64_t)gy * W + gx];
      }
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int c = threadIdx.x + i * kBlock;
      if (c < kMorphF * kMorphF) buf[0][(c / kMorphF) * kMorphP + c % kMorphF] = v[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 1; k <= 4; ++k) {
    const uint8_t* src = buf[(k - 1) & 1];
    uint8_t* dst = buf[k & 1];
    const int os = (1 - k) & 3, od = (-k) & 3;   // byte offsets of frame column 0
    const bool mx = k == 2 || k == 3;
    constexpr int kMaxGroups = (kMorphF - 2 + 3) / 4;
    const int n = kMorphF - 2 * k, ng = (n + 3) / 4;
    for (int c = threadIdx.x; c < n * kMaxGroups; c += kBlock) {
      const int fy = k + c / kMaxGroups, g = c % kMaxGroups;
      if (g >= ng) continue;
      const int fx = k + 4 * g;
      uint32_t h[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const uint32_t* q = (const uint32_t*)(src + (fy - 1 + j) * kMorphP + fx - 1 + os);
        const uint32_t a = q[0], b = q[1];
        const uint32_t l = a, m = __builtin_amdgcn_alignbyte(b, a, 1), r = __builtin_amdgcn_alignbyte(b, a, 2);
        h[j] = mx ? max4(max4(l, m), r) : min4(min4(l, m), r);
      }
      const uint32_t o = mx ? max4(max4(h[0], h[1]), h[2]) : min4(min4(h[0], h[1]), h[2]);
      *(uint32_t*)(dst + fy * kMorphP + fx + od) = o;
    }
    __syncthreads();
    if (edge) {
      // the box's cells outside the image take the nearest cell inside
      for (int c = threadIdx.x; c < n * n; c += kBlock) {
        const int fy = k + c / n, fx = k + c % n;
        const int gy = y0 + fy, gx = x0 + fx;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) continue;
        const int cy = min(max(gy, 0), H - 1) - y0, cx = min(max(gx, 0), W - 1) - x0;
        dst[fy * kMorphP + fx + od] = dst[cy * kMorphP + cx + od];
      }
      __syncthreads();
    }
  }
  // boundary of the tile from the closed labels (buf[0], offset 0)
  const uint8_t* lb = buf[0];
  constexpr int kTileGroups = kMorphT / 4;
  for (int c = threadIdx.x; c < kMorphT * kTileGroups; c += kBlock) {
    const int ty = c / kTileGroups, g = c % kTileGroups;
    const int fy = kMorphHalo + ty, fx = kMorphHalo + 4 * g;
    uint32_t nb[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const uint32_t* q = (const uint32_t*)(lb + (fy - 1 + j) * kMorphP + fx - 1);
      const uint32_t a = q[0], b = q[1];
      nb[j][0] = a; nb[j][1] = __builtin_amdgcn_alignbyte(b, a, 1); nb[j][2] = __builtin_amdgcn_alignbyte(b, a, 2);
    }
    const uint32_t v = nb[1][1];
    uint32_t acc = 0u;   // bit 7 of a byte: some neighbour differs
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        if (j != 1 || i != 1) acc |= ((nb[j][i] ^ v) + 0x7F7F7F7Fu) & 0x80808080u;
    const uint32_t r = (acc >> 7) & 0x01010101u;
    const int gy = y0 + fy, gx = x0 + fx;   // gx a multiple of 4
    if (wide) {
      *(uint32_t*)(B + (int64_t)gy * W + gx) = r;
      if (closed) *(uint32_t*)(closed + (int64_t)gy * W + gx) = v;
      continue;
    }
    if (gy >= H) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = gx + j;
      if (x >= W) break;
      uint8_t bj = (uint8_t)(r >> (8 * j));
      if (gy == 0 || gy == H - 1 || x == 0 || x == W - 1) {
        // on the image's border: neighbours outside the image do not count
        const uint8_t* q = lb + fy * kMorphP + fx + j;
        const int cv = q[0];
        bool d = false;
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx)
            if ((dy || dx) && gy + dy >= 0 && gy + dy < H && x + dx >= 0 && x + dx < W)
              d |= q[dy * kMorphP + dx] != cv;
        bj = d ? 1 : 0;
      }
      B[(int64_t)gy * W + x] = bj;
      if (closed) closed[(int64_t)gy * W + x] = (uint8_t)(v >> (8 * j));
    }
  }
}

// The paper's refinement in one pass over the image: the Moore boundary of
// the labels, then 'fill', then 'remove', per tile of kMorphT x kMorphT
// pixels with a 3-pixel halo in LDS, four cells per thread and step as in
// k_morph_refine (the maps after the first step hold 0 and 1, so 'fill' and
// 'remove' are plain bitwise ands and ors of neighbour words). The boundary
// step ignores neighbours outside the image (cells on the image's border
// rows and columns are taken again without them); 'fill' and 'remove' take
// them as 0, so at an image edge every step's cells outside the image are
// set to 0 before the next step reads them.
constexpr int kPaperHalo = 3, kPaperF = kMorphT + 2 * kPaperHalo;   // frame: 70 x 70
__global__ __launch_bounds__(kBlock) void k_paper_refine(const uint8_t* __restrict__ lab, int32_t W, int32_t H,
                                                         uint8_t* __restrict__ B, int32_t words) {
  __shared__ __attribute__((aligned(16))) uint8_t buf[2][kPaperF * kMorphP];
  const int x0 = blockIdx.x * kMorphT - kPaperHalo, y0 = blockIdx.y * kMorphT - kPaperHalo;   // frame origin
  const bool edge = x0 < 0 || y0 < 0 || x0 + kPaperF > W || y0 + kPaperF > H;
  const bool wide = !edge && words;
  auto inside = [&](int gy, int gx) { return gy >= 0 && gy < H && gx >= 0 && gx < W; };
  if (wide) {
    constexpr int kWords = (kPaperF + 1 + 3) / 4;   // global words covering a frame row from column x0 - 1
    for (int c = threadIdx.x; c < kPaperF * kWords; c += kBlock) {
      const int fy = c / kWords, w = c - fy * kWords;
      const uint8_t* row = lab + (int64_t)(y0 + fy) * W;
      const int g0 = x0 - 1 + 4 * w;   // a multiple of 4 (x0 = 64 bx - 3)
      uint32_t v = 0u;
      if (g0 + 3 < W) v = *(const uint32_t*)(row + g0);
      else
        for (int j = 0; j < 4; ++j)
          if (g0 + j < W) v |= (uint32_t)row[g0 + j] << (8 * j);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int fx = 4 * w + j - 1;
        if (fx >= 0 && fx < kPaperF) buf[0][fy * kMorphP + fx] = (uint8_t)(v >> (8 * j));
      }
    }
  } else {
    constexpr int kPer = (kPaperF * kPaperF + kBlock - 1) / kBlock;
    uint8_t v[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int c = threadIdx.x + i * kBlock;
      v[i] = 0;
      if (c < kPaperF * kPaperF) {
        const int fy = c / kPaperF, fx = c - fy * kPaperF;
        const int gy = min(max(y0 + fy, 0), H - 1), gx = min(max(x0 + fx, 0), W - 1);
        v[i] = lab[(int64_t)gy * W + gx];
      }
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int c = threadIdx.x + i * kBlock;
      if (c < kPaperF * kPaperF) buf[0][(c / kPaperF) * kMorphP + c % kPaperF] = v[i];
    }
  }
  __syncthreads();
  // the three neighbour words (left, centre, right) of a row of four cells
  auto row3 = [&](const uint8_t* p, uint32_t& l, uint32_t& m, uint32_t& r) {
    const uint32_t a = ((const uint32_t*)p)[0], b = ((const uint32_t*)p)[1];
    l = a; m = __builtin_amdgcn_alignbyte(b, a, 1); r = __builtin_amdgcn_alignbyte(b, a, 2);
  };
  // steps 1 and 2 on the frame inset by k (k = 1: boundary, k = 2: fill); offsets as in k_morph_refine
#pragma unroll
  for (int k = 1; k <= 2; ++k) {
    const uint8_t* src = buf[(k - 1) & 1];
    uint8_t* dst = buf[k & 1];
    const int os = (1 - k) & 3, od = (-k) & 3;
    constexpr int kMaxGroups = (kPaperF - 2 + 3) / 4;
    const int n = kPaperF - 2 * k, ng = (n + 3) / 4;
    for (int c = threadIdx.x; c < n * kMaxGroups; c += kBlock) {
      const int fy = k + c / kMaxGroups, g = c % kMaxGroups;
      if (g >= ng) continue;
      const int fx = k + 4 * g;
      uint32_t nb[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j) row3(src + (fy - 1 + j) * kMorphP + fx - 1 + os, nb[j][0], nb[j][1], nb[j][2]);
      const uint32_t v = nb[1][1];
      uint32_t o;
      if (k == 1) {
        uint32_t acc = 0u;   // bit 7 of a byte: some neighbour differs (labels < 128)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int i = 0; i < 3; ++i)
            if (j != 1 || i != 1) acc |= ((nb[j][i] ^ v) + 0x7F7F7F7Fu) & 0x80808080u;
        o = (acc >> 7) & 0x01010101u;
      } else {
        uint32_t all = 0x01010101u;   // every neighbour 1
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int i = 0; i < 3; ++i)
            if (j != 1 || i != 1) all &= nb[j][i];
        o = v | all;
      }
      *(uint32_t*)(dst + fy * kMorphP + fx + od) = o;
    }
    __syncthreads();
    if (edge) {
      for (int c = threadIdx.x; c < n * n; c += kBlock) {
        const int fy = k + c / n, fx = k + c % n;
        const int gy = y0 + fy, gx = x0 + fx;
        uint8_t* d = dst + fy * kMorphP + fx + od;
        if (!inside(gy, gx)) { *d = 0; continue; }   // outside: 0 for the steps that follow
        if (k == 1 && (gy == 0 || gy == H - 1 || gx == 0 || gx == W - 1)) {
          // on the image's border: the boundary without the neighbours outside
          const uint8_t* q = src + fy * kMorphP + fx + os;
          const int cv = q[0];
          bool diff = false;
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
              if ((dy || dx) && inside(gy + dy, gx + dx)) diff |= q[dy * kMorphP + dx] != cv;
          *d = diff ? 1 : 0;
        }
      }
      __syncthreads();
    }
  }
  // step 3: 'remove' on the tile, from buf[0] (offset 2)
  constexpr int kTileGroups = kMorphT / 4;
  for (int c = threadIdx.x; c < kMorphT * kTileGroups; c += kBlock) {
    const int ty = c / kTileGroups, g = c % kTileGroups;
    const int fy = kPaperHalo + ty, fx = kPaperHalo + 4 * g;
    uint32_t u, l, v, r, dn, t0, t1;
    row3(buf[0] + (fy - 1) * kMorphP + fx - 1 + 2, t0, u, t1);
    row3(buf[0] + fy * kMorphP + fx - 1 + 2, l, v, r);
    row3(buf[0] + (fy + 1) * kMorphP + fx - 1 + 2, t0, dn, t1);
    const uint32_t o = v & ~(u & dn & l & r);
    const int gy = y0 + fy, gx = x0 + fx;   // gx a multiple of 4
    if (wide) {
      *(uint32_t*)(B + (int64_t)gy * W + gx) = o;
      continue;
    }
    if (gy >= H) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (gx + j < W) B[(int64_t)gy * W + gx + j] = (uint8_t)(o >> (8 * j));
  }
}

// ---------------------------------------------------------------------------
// Connected components by union-find. A link always points a larger root at
// a smaller one, so a component's root ends as its smallest index.
// Root of a, halving the path on the way (each visited pixel is pointed at
// its grandparent with an atomic minimum, so a link only ever moves towards
// smaller indices of the same component).
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t a) {
  for (;;) {
    const int32_t p = __hip_atomic_load(&parent[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == a) return a;
    const int32_t pp = __hip_atomic_load(&parent[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (pp == p) return p;
    atomicMin(&parent[a], pp);
    a = pp;
  }
}

__device__ __forceinline__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
  for (;;) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) { const int32_t t = a; a = b; b = t; }
    // a > b, a was a root when found: make it point at b unless it moved meanwhile
    const int32_t old = atomicMin(&parent[a], b);
    if (old == a) return;
    a = old;   // a was linked elsewhere concurrently: continue from there
  }
}

// Two-level merge. k_cc_tile: one block per tile of kTileW x kTileH pixels
// runs the same union-find on the tile's pixels in LDS (links from larger to
// smaller local raster index, which is the global raster order within the
// tile), then writes for every pixel of the tile the global index of its
// tile root (-1 off the boundary map) and the tile roots' local sizes (0
// elsewhere), which initialises the whole forest. k_cc_edges then unions, through the global forest, only the
// neighbour pairs that cross a tile edge. The forest's roots stay the
// smallest raster index of their component.
constexpr int kTileW = 64, kTileH = 32;
static_assert(kTileW == 64, "k_cc_tile: one wavefront per tile row");
static_assert(kTileW + 2 * (kTileH - 1) <= 128, "k_cc_edges: one thread per tile edge pixel");

__device__ __forceinline__ int32_t lds_find(int32_t* lp, int32_t a) {
  for (;;) {
    const int32_t p = lp[a];
    if (p == a) return a;
    const int32_t pp = lp[p];
    if (pp == p) return p;
    atomicMin(&lp[a], pp);
    a = pp;
  }
}

__device__ __forceinline__ void lds_union(int32_t* lp, int32_t a, int32_t b) {
  for (;;) {
    a = lds_find(lp, a);
    b = lds_find(lp, b);
    if (a == b) return;
    if (a < b) { const int32_t t = a; a = b; b = t; }
    const int32_t old = atomicMin(&lp[a], b);
    if (old == a) return;
    a = old;
  }
}

__global__ __launch_bounds__(kBlock) void k_cc_tile(const uint8_t* __restrict__ B, int32_t W, int32_t H,
                                                    int32_t* parent, int32_t* size) {
  __shared__ int32_t lp[kTileW * kTileH];
  __shared__ int32_t lsz[kTileW * kTileH];
  const int x0 = blockIdx.x * kTileW, y0 = blockIdx.y * kTileH;
  const int lx = threadIdx.x & (kTileW - 1);
  constexpr int kRowsPerPass = kBlock / kTileW;
  // wavefront w takes the band of rows w kBand .. w kBand + kBand - 1, one
  // row per pass, so a row's upward unions meet a row its own wavefront
  // linked one pass before (short paths to the roots)
  constexpr int kBand = kTileH / kRowsPerPass;
  bool on[kTileH / kRowsPerPass], first[kTileH / kRowsPerPass];
#pragma unroll
  for (int j = 0; j < kTileH / kRowsPerPass; ++j) {
    const int ly = (int)(threadIdx.x / kTileW) * kBand + j;
    const int x = x0 + lx, y = y0 + ly;
    on[j] = x < W && y < H && B[(int64_t)y * W + x] != 0;
    // a wavefront holds one tile row (kTileW == 64): each pixel links
    // straight to the first pixel of its horizontal run, so left neighbours
    // need no union below
    const uint64_t row = __builtin_amdgcn_ballot_w64(on[j]);
    const uint64_t upto = lx == 63 ? ~0ull : ((2ull << lx) - 1ull);   // bits 0 .. lx
    const uint64_t gaps = ~row & upto;
    const int start = gaps ? 64 - __builtin_clzll(gaps) : 0;   // just past the last gap at or before lx
    first[j] = start == lx;
    lp[ly * kTileW + lx] = on[j] ? ly * kTileW + start : -1;
    lsz[ly * kTileW + lx] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kTileH / kRowsPerPass; ++j) {
    if (!on[j]) continue;
    const int ly = (int)(threadIdx.x / kTileW) * kBand + j;
    const int l = ly * kTileW + lx;
    // the tile's neighbours before this pixel in raster order (8-connectivity;
    // the left one is in its run already). Above: one union per horizontal
    // run of the row above that touches the pixel and not the pixel before
    // it in its own run (those are joined through that pixel already), so
    // a run's first pixel takes the first pixel of each run among its three
    // upper neighbours, every later pixel only a run starting up-right.
    if (ly > 0) {
      const int u = l - kTileW;
      const bool ul = lx > 0 && lp[u - 1] >= 0, uc = lp[u] >= 0, ur = lx + 1 < kTileW && lp[u + 1] >= 0;
      if (first[j]) {
        if (ul) lds_union(lp, l, u - 1);
        if (uc && !ul) lds_union(lp, l, u);
      }
      if (ur && !uc) lds_union(lp, l, u + 1);
    }
  }
  __syncthreads();
  // every pixel of the tile gets its parent (-1 off the boundary map), so no
  // separate pass initialises the forest
#pragma unroll
  for (int j = 0; j < kTileH / kRowsPerPass; ++j) {
    const int ly = (int)(threadIdx.x / kTileW) * kBand + j;
    if (x0 + lx >= W || y0 + ly >= H) continue;
    int32_t gp = -1;
    if (on[j]) {
      const int32_t r = lds_find(lp, ly * kTileW + lx);
      gp = (y0 + r / kTileW) * W + x0 + (r % kTileW);
      atomicAdd(&lsz[r], 1);
    }
    parent[(int64_t)(y0 + ly) * W + x0 + lx] = gp;
  }
  __syncthreads();
  // each tile root's local component size, at the root (0 everywhere else)
#pragma unroll
  for (int j = 0; j < kTileH / kRowsPerPass; ++j) {
    const int ly = (int)(threadIdx.x / kTileW) * kBand + j;
    const int l = ly * kTileW + lx;
    if (x0 + lx < W && y0 + ly < H) size[(int64_t)(y0 + ly) * W + x0 + lx] = on[j] ? lsz[l] : 0;
  }
}

// Neighbour pairs across tile edges: thread t of a tile's block takes edge
// pixel t (its top row, then its left and right columns below the top row).
// Along the top row the rule of k_cc_tile applies: the row's runs are joined
// inside the tile already and so are the runs of the row above (inside its
// tiles, or by the left-column unions of the tile holding their right part),
// so a run's first pixel takes up-left, and up when up-left is off, and every
// pixel takes up-right only when up is off.
__global__ __launch_bounds__(128) void k_cc_edges(const uint8_t* __restrict__ B, int32_t W, int32_t H,
                                                  int32_t* parent) {
  const int x0 = blockIdx.x * kTileW, y0 = blockIdx.y * kTileH;
  const int t = threadIdx.x;
  int lx = 0, ly = 0;
  if (t < kTileW) { lx = t; ly = 0; }
  else if (t < kTileW + kTileH - 1) { lx = 0; ly = t - kTileW + 1; }
  else if (t < kTileW + 2 * (kTileH - 1)) { lx = kTileW - 1; ly = t - kTileW - kTileH + 2; }
  const int x = x0 + lx, y = y0 + ly;
  const bool in = t < kTileW + 2 * (kTileH - 1) && x < W && y < H;
  const int32_t i = y * W + x;
  const bool on = in && B[i] != 0;
  bool first = true;
  if (t < kTileW) {   // wavefront 0 holds the top row (kTileW == 64)
    const uint64_t row = __builtin_amdgcn_ballot_w64(on);
    first = lx == 0 || ((row >> (lx - 1)) & 1ull) == 0;
  }
  if (!on) return;
  // raster-earlier neighbours that lie in another tile
  if (x > 0 && lx == 0 && B[i - 1]) uf_union(parent, i, i - 1);
  if (y > 0) {
    const int32_t u = i - W;
    if (ly == 0) {
      const bool ul = x > 0 && B[u - 1], uc = B[u] != 0, ur = x + 1 < W && B[u + 1];
      if (first) {
        if (ul) uf_union(parent, i, u - 1);
        if (uc && !ul) uf_union(parent, i, u);
      }
      if (ur && !uc) uf_union(parent, i, u + 1);
    } else {
      if (lx == 0 && x > 0 && B[u - 1]) uf_union(parent, i, u - 1);
      if (lx == kTileW - 1 && x + 1 < W && B[u + 1]) uf_union(parent, i, u + 1);
    }
  }
}

// Roots for every pixel (plain loads: the forest is final), and component
// sizes at the roots: k_cc_tile left each tile root's local size at the tile
// root; a tile root that is not its component's root moves its count to the
// root with one atomic. Roots of components are always tile roots (a
// component's smallest index is the smallest of its tile part), so no count
// moves into a tile root that moves its own count away.
__global__ __launch_bounds__(kBlock) void k_cc_flatten(int64_t N, int32_t* parent, int32_t* size) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    if (parent[i] < 0) continue;
    // No link changes after the merge kernels except pixels being pointed at
    // their root here, so any value read (cached, possibly stale) is an
    // ancestor of i and the walk ends at i's root.
    const int32_t t = parent[i];   // its tile root (or, for tile-edge pixels, an ancestor of it)
    int32_t r = t;
    for (int32_t q = parent[r]; q != r; q = parent[r]) r = q;
    parent[i] = r;
    if (t != r) parent[t] = r;     // shortcut: the tile's other pixels reach r in two steps
    if (r != (int32_t)i) {
      const int32_t sz = size[i];
      if (sz > 0) {
        size[i] = 0;
        atomicAdd(&size[r], sz);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Paper filter: components in ascending (size, root) order are dropped while
// the dropped total stays <= floor(0.04 * total). With cnt[s] the number of
// components of size s (s <= budget), everything below the first size s* that
// no longer fits whole is dropped, and of size s* the first m by root.
struct DropRule {
  long long total;    // boundary pixels
  long long budget;   // floor(drop_frac * total)
  int32_t s_star;     // sizes < s_star dropped; 0: none
  int32_t m;          // components of size s_star dropped (smallest roots first)
};

// cnt[s] += 1 for every component of size s; total = all boundary pixels.
__global__ __launch_bounds__(kBlock) void k_drop_count(const int32_t* __restrict__ size, int64_t N,
                                                       unsigned long long* total, int32_t* cnt) {
  constexpr int kSmall = 1024;   // sizes below this are counted per block in LDS first
  __shared__ unsigned long long part;
  __shared__ int32_t small[kSmall];
  for (int j = threadIdx.x; j < kSmall; j += blockDim.x) small[j] = 0;
  if (threadIdx.x == 0) part = 0;
  __syncthreads();
  unsigned long long mine = 0;
  // After k_cc_flatten a pixel's size is non-zero exactly at the roots
  // (tile roots that are not roots handed their counts on and hold 0).
  auto count_root = [&](int32_t s) {
    if (s <= 0) return;
    mine += (unsigned long long)s;
    if (s < kSmall) atomicAdd(&small[s], 1);
    else atomicAdd(&cnt[s], 1);
  };
  // four pixels per thread and step (one 16-byte load of sizes: the grid is
  // small, so each thread needs several loads in flight), then the tail
  const int64_t nq = N >> 2;
  const int4* sq = (const int4*)size;   // 16-byte aligned: in the 256-byte aligned workspace
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
    const int4 v = sq[q];
    count_root(v.x);
    count_root(v.y);
    count_root(v.z);
    count_root(v.w);
  }
  if (blockIdx.x == 0)
    for (int64_t i = (nq << 2) + threadIdx.x; i < N; i += blockDim.x) count_root(size[i]);
  // one LDS add per wavefront (adds to one word from every lane serialise)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off, 64);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&part, mine);
  __syncthreads();
  for (int j = threadIdx.x; j < kSmall && j <= N; j += blockDim.x)
    if (small[j]) atomicAdd(&cnt[j], small[j]);
  if (threadIdx.x == 0) atomicAdd(total, part);
}

// One block: the budget floor(drop_frac * total) (the rule's comparison in
// fp64), then a walk over sizes 1..budget in order, a block-wide scan per
// chunk of 1024 sizes, to the first size that does not fit whole.
__global__ __launch_bounds__(1024) void k_drop_find(const int32_t* __restrict__ cnt,
                                                    const unsigned long long* __restrict__ total, double drop_frac,
                                                    DropRule* rule) {
  __shared__ unsigned long long sc[1024];
  __shared__ int done;
  __shared__ unsigned long long base_s;
  const unsigned long long t = *total;
  const long long bud = (long long)floor(drop_frac * (double)t);
  if (threadIdx.x == 0) {
    done = 0;
    base_s = 0;
    rule->total = (long long)t;
    rule->budget = bud;
    rule->s_star = (int32_t)(bud + 1);   // every size <= budget fits: the first size > budget stops the walk
    rule->m = 0;
  }
  __syncthreads();
  for (long long s0 = 1; s0 <= bud; s0 += 1024) {
    const long long s = s0 + threadIdx.x;
    const unsigned long long w = s <= bud ? (unsigned long long)cnt[s] * (unsigned long long)s : 0ull;
    sc[threadIdx.x] = w;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const unsigned long long a = threadIdx.x >= off ? sc[threadIdx.x - off] : 0ull;
      __syncthreads();
      sc[threadIdx.x] += a;
      __syncthreads();
    }
    const unsigned long long below = base_s + sc[threadIdx.x] - w;   // pixels of all sizes < s
    // s is the first size that does not fit whole: below fits, below + w does not
    if (s <= bud && below + w > (unsigned long long)bud && below <= (unsigned long long)bud) {
      // exactly one thread can see this (the running total crosses once)
      rule->s_star = (int32_t)s;
      rule->m = (int32_t)(((unsigned long long)bud - below) / (unsigned long long)s);
      done = 1;
    }
    __syncthreads();
    if (done) break;
    if (threadIdx.x == 1023) base_s += sc[1023];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of 0/1 flags in three launches: per-block
// counts, a scan of the counts in one block, then per-block prefix and
// scatter. Flag sources:
//   kind 0 (roots of size s*):  rank[i] = number of such roots before i
//   kind 1 (list):              out[pos] = i for border columns and kept pixels
// Fraction control (a benchmark knob, not the paper's): exactly `want`
// pixels ranked as (1) border columns by raster index, (2) kept pixels by
// component size descending, then raster index, (3) all other pixels by
// chessboard distance to (1)+(2) ascending, then h(i) = mix64(i ^ seed), then
// raster index. The selection is threshold-based: a radix select finds the
// key of the want-th pixel within the class it falls in, ties at that key go
// by raster order (a device-wide scan).
struct RadixSel {
  unsigned long long prefix;   // key bits found so far (top digits first)
  long long need;              // rank (1-based) of the wanted key among the candidates
  long long below;             // candidates with a smaller key (of the digits fixed so far)
};

struct FracState {
  long long want, n0, n1;
  int32_t mode;                // 0: border only, 1: + kept pixels, 2: + other pixels
  RadixSel s1;                 // kept pixels: key ~size (size descending)
  RadixSel s2;                 // other pixels: key distance
  RadixSel s3;                 // other pixels at distance s2.prefix: key h(i)
};

struct ScanCtx {
  const uint8_t* B;       // boundary map after refinement
  const int32_t* parent;  // flattened: root of each boundary pixel, -1 elsewhere
  const int32_t* size;    // size at roots
  const DropRule* rule;   // paper filter (nullptr: configured filter)
  int64_t min_cc;
  int32_t W;
  int64_t N;
  int32_t* rank;          // kind 0 output
  uint32_t* out;          // kind 1 output
  uint8_t* refined;       // kind 1 optional output: kept map
  long long* count;       // kind 1: list length
  const FracState* fc;    // fraction control (nullptr: list = border columns + kept pixels)
  const int32_t* dist;    // chessboard distance to border + kept pixels
  int32_t* frank;         // kinds 2, 3 output: rank of a tie in raster order
  unsigned long long seed;
  const uint8_t* cls;     // fraction control: 0 border column, 1 kept, 2 other
  // The flags of a scan, one bit per element (word i >> 6, bit i & 63):
  // written by the counting pass, read by the applying pass instead of
  // working the flags out again (nullptr: both passes work them out).
  unsigned long long* bits;
};

// Kept: the pixel's component (root r, -1 for no boundary pixel) passes the filter.
__device__ __forceinline__ bool kept_root(const ScanCtx& c, int32_t r) {
  if (r < 0) return false;
  const int32_t s = c.size[r];
  if (!c.rule) return s >= c.min_cc;
  if (s < c.rule->s_star) return false;
  if (s == c.rule->s_star) return c.rank[r] >= c.rule->m;
  return true;
}
__device__ __forceinline__ bool kept(const ScanCtx& c, int64_t i) { return kept_root(c, c.parent[i]); }

// SplitMix64's output function (Steele, Lea and Flood; constants as
// published by Vigna), on the raster index xor the seed.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ bool border(const ScanCtx& c, int64_t i) {
  const int x = (int)((uint32_t)i % (uint32_t)c.W);   // W * H < 2^31: 32-bit division suffices
  return x == 0 || x == c.W - 1;
}

__device__ __forceinline__ int32_t comp_size(const ScanCtx& c, int64_t i) { return c.size[c.parent[i]]; }

__device__ __forceinline__ bool selected(const ScanCtx& c, int64_t i) {
  const bool b = border(c, i);
  if (!c.fc) return b || kept(c, i);
  const FracState& f = *c.fc;
  if (f.mode == 0) {
    if (!b) return false;
    const int64_t y = (uint32_t)i / (uint32_t)c.W;
    const int64_t rank0 = c.W == 1 ? y : 2 * y + (((uint32_t)i % (uint32_t)c.W) == (uint32_t)(c.W - 1) ? 1 : 0);
    return rank0 < f.want;
  }
  if (b) return true;
  const bool k = c.cls[i] == 1;
  if (f.mode == 1) {
    if (!k) return false;
    const uint32_t key = ~(uint32_t)comp_size(c, i);
    const uint32_t kstar = (uint32_t)f.s1.prefix;
    return key < kstar || (key == kstar && c.frank[i] < f.s1.need - f.s1.below);
  }
  if (k) return true;
  const uint32_t d = (uint32_t)c.dist[i], dstar = (uint32_t)f.s2.prefix;
  if (d != dstar) return d < dstar;
  const unsigned long long h = mix64((unsigned long long)i ^ c.seed);
  return h < f.s3.prefix || (h == f.s3.prefix && c.frank[i] < f.s3.need - f.s3.below);
}

template <int KIND>
__device__ __forceinline__ bool flag(const ScanCtx& c, int64_t i) {
  if constexpr (KIND == 0) {
    return c.parent[i] == (int32_t)i && c.size[i] == c.rule->s_star;
  } else if constexpr (KIND == 1) {
    return selected(c, i);
  } else if constexpr (KIND == 2) {   // kept, not border, size at the threshold
    return c.cls[i] == 1 && ~(uint32_t)comp_size(c, i) == (uint32_t)c.fc->s1.prefix;
  } else {                            // other pixels at the threshold distance and hash
    return c.cls[i] == 2 && (uint32_t)c.dist[i] == (uint32_t)c.fc->s2.prefix &&
           mix64((unsigned long long)i ^ c.seed) == c.fc->s3.prefix;
  }
}

// Inclusive scan of one value per lane across the wavefront (shuffles).
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t a = (uint32_t)__shfl_up((int)v, off);
    if (lane >= off) v += a;
  }
  return v;
}

// Exclusive scan of the per-lane values of a block of kWaves wavefronts:
// wavefront scans, then the wavefront totals through LDS (two barriers).
template <int kWaves>
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* wtot, uint32_t& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t incl = wave_scan_incl(v);
  if (lane == 63) wtot[wv] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int j = 0; j < kWaves; ++j) {
    const uint32_t t = wtot[j];
    before += j < wv ? t : 0u;
    all += t;
  }
  __syncthreads();   // wtot may be rewritten after this
  total = all;
  return before + incl - v;
}

template <int KIND>
__global__ __launch_bounds__(kBlock) void k_scan_count(ScanCtx c, uint32_t* bsum) {
  __shared__ uint32_t s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * kScanPer;
  uint32_t m = 0;
#pragma unroll
  for (int j0 = 0; j0 < kScanPer; j0 += kBlock) {
    const int64_t i = i0 + j0 + threadIdx.x;
    const bool fl = i < c.N && flag<KIND>(c, i);
    m += fl;
    if (c.bits) {
      // the wavefront's 64 consecutive elements as one word
      const unsigned long long w = __builtin_amdgcn_ballot_w64(fl);
      if ((threadIdx.x & 63) == 0) c.bits[(i0 + j0 + threadIdx.x) >> 6] = w;
    }
  }
  m = wave_scan_incl(m);   // lane 63: the wavefront's count
  if ((threadIdx.x & 63) == 63) atomicAdd(&s, m);
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

// exclusive scan of nb block counts in place (one block of 1024 threads):
// the counts are read into LDS with coalesced loads (up to kTopLds of them;
// beyond that straight from global memory), each thread sums a contiguous
// run of them, the runs are scanned across the block, then each thread
// writes its run's prefixes back to LDS and the block stores them coalesced.
constexpr int kTopLds = 12288;   // 48 KB: 4096x3072 pixels at 1024 per count
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* bsum, int64_t nb, long long* total) {
  __shared__ uint32_t wtot[16];
  __shared__ uint32_t v[kTopLds];
  const bool in_lds = nb <= kTopLds;
  if (in_lds)
    for (int64_t b = threadIdx.x; b < nb; b += 1024) v[b] = bsum[b];
  __syncthreads();
  uint32_t* src = in_lds ? v : bsum;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = min(b0 + per, nb);
  uint32_t run = 0;
  for (int64_t b = b0; b < b1; ++b) run += src[b];
  uint32_t all;
  uint32_t pos = block_scan_excl<16>(run, wtot, all);   // (its barriers order the reads above before the writes below)
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t c = src[b];
    src[b] = pos;
    pos += c;
  }
  if (in_lds) {
    __syncthreads();
    for (int64_t b = threadIdx.x; b < nb; b += 1024) bsum[b] = v[b];
  }
  if (threadIdx.x == 0 && total) *total = (long long)all;
}

template <int KIND>
__global__ __launch_bounds__(kBlock) void k_scan_apply(ScanCtx c, const uint32_t* bsum) {
  // thread t owns elements i0 + per t .. i0 + per t + per - 1 (in order)
  __shared__ uint32_t sc[kBlock / 64];
  const int64_t i0 = (int64_t)blockIdx.x * kScanPer;
  constexpr int per = kScanPer / kBlock;
  static_assert(64 % per == 0, "a thread's flags lie in one word");
  bool f[per];
  uint32_t m = 0;
  if (c.bits) {
    const int64_t e = i0 + (int64_t)threadIdx.x * per;   // per divides 64: one word holds the thread's flags
    const unsigned long long w = c.bits[e >> 6] >> (e & 63);
#pragma unroll
    for (int j = 0; j < per; ++j) {
      f[j] = (w >> j) & 1ull;
      m += f[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < per; ++j) {
      const int64_t i = i0 + (int64_t)threadIdx.x * per + j;
      f[j] = i < c.N && flag<KIND>(c, i);
      m += f[j];
    }
  }
  uint32_t all;
  uint32_t pos = bsum[blockIdx.x] + block_scan_excl<kBlock / 64>(m, sc, all);
#pragma unroll
  for (int j = 0; j < per; ++j) {
    const int64_t i = i0 + (int64_t)threadIdx.x * per + j;
    if (i >= c.N) break;
    if constexpr (KIND == 0) {
      if (f[j]) c.rank[i] = (int32_t)pos;
    } else if constexpr (KIND == 1) {
      if (f[j]) c.out[pos] = (uint32_t)i;
      if (c.refined) c.refined[i] = kept(c, i) ? 1 : 0;
    } else {
      if (f[j]) c.frank[i] = (int32_t)pos;
    }
    pos += f[j];
  }
}

// ---------------------------------------------------------------------------
// Fraction control kernels.
// Class of every pixel (0 border column, 1 kept, 2 other) and the kept count.
// Class of every pixel: 0 border column, 1 kept, 2 other; and the count of
// kept pixels. Four pixels per thread and step: one 16-byte load of their
// parents, one word of classes written (the workspace keeps both arrays
// 256-byte aligned), the column of the first one divided out once.
__global__ __launch_bounds__(kBlock) void k_fc_class(ScanCtx c, uint8_t* cls, unsigned long long* n1) {
  __shared__ unsigned long long part;
  if (threadIdx.x == 0) part = 0;
  __syncthreads();
  unsigned long long mine = 0;
  auto cls_of = [&](int x, int32_t r) -> uint32_t {
    return (x == 0 || x == c.W - 1) ? 0u : (kept_root(c, r) ? 1u : 2u);
  };
  // the filter's fields once; the four component sizes of a quad gathered
  // together (from index 0 for pixels without a component), so a quad costs
  // two round trips to memory, not five
  const bool rule = c.rule != nullptr;
  const int32_t s_star = rule ? c.rule->s_star : 0, m_star = rule ? c.rule->m : 0;
  const int64_t nq = c.N >> 2;
  const int4* pq = (const int4*)c.parent;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
    const int4 p = pq[q];
    int x = (int)((uint32_t)(q << 2) % (uint32_t)c.W);   // W * H < 2^31: 32-bit division suffices
    const int32_t r[4] = {p.x, p.y, p.z, p.w};
    int32_t sz[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) sz[b] = c.size[r[b] < 0 ? 0 : r[b]];
    uint32_t w = 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      bool kp = r[b] >= 0;
      if (kp) {
        if (!rule) kp = sz[b] >= c.min_cc;
        else kp = sz[b] > s_star || (sz[b] == s_star && c.rank[r[b]] >= m_star);
      }
      const uint32_t k = (x == 0 || x == c.W - 1) ? 0u : (kp ? 1u : 2u);
      w |= k << (8 * b);
      mine += k == 1u ? 1ull : 0ull;
      x = x + 1 == c.W ? 0 : x + 1;
    }
    ((uint32_t*)cls)[q] = w;
  }
  if (blockIdx.x == 0)
    for (int64_t i = (nq << 2) + threadIdx.x; i < c.N; i += blockDim.x) {
      const uint32_t k = cls_of((int)((uint32_t)i % (uint32_t)c.W), c.parent[i]);
      cls[i] = (uint8_t)k;
      mine += k == 1u ? 1ull : 0ull;
    }
  // one LDS add per wavefront (adds to one word from every lane serialise)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off, 64);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&part, mine);
  __syncthreads();
  // one of kN1Parts counters per block: adds to a single word from thousands
  // of blocks queue up one after another at the memory side
  if (threadIdx.x == 0 && part) atomicAdd(&n1[blockIdx.x % kN1Parts], part);
}

// Which class the want-th pixel falls in, and the rank wanted inside it.
__global__ void k_fc_plan(FracState* f, const unsigned long long* n1, long long want, long long n0,
                          unsigned long long s1_prefix) {
  f->want = want;
  f->n0 = n0;
  long long nk = 0;
  for (int k = 0; k < kN1Parts; ++k) nk += (long long)n1[k];
  f->n1 = nk;
  f->s1 = RadixSel{s1_prefix, 0, 0};
  f->s2 = RadixSel{0, 0, 0};
  f->s3 = RadixSel{0, 0, 0};
  if (f->want <= f->n0) { f->mode = 0; return; }
  if (f->want <= f->n0 + f->n1) { f->mode = 1; f->s1.need = f->want - f->n0; return; }
  f->mode = 2;
  f->s2.need = f->want - f->n0 - f->n1;
}

// The rank wanted at distance s2.prefix among the other pixels.
__global__ void k_fc_after_dist(FracState* f) { f->s3 = RadixSel{0, f->s2.need - f->s2.below, 0}; }

// Radix select, one 8-bit digit per pass from the top: per-block digit
// histograms of the candidates whose higher digits match, then one block
// picks the digit where the running count reaches `need`.
template <int SEL>
__device__ __forceinline__ bool rs_key(const ScanCtx& c, int64_t i, unsigned long long& key) {
  if constexpr (SEL == 1) {
    if (c.cls[i] != 1) return false;
    key = ~(uint32_t)comp_size(c, i);
  } else {
    static_assert(SEL == 2, "the hash select runs over compacted candidates (k_rs_hist_cands)");
    if (c.cls[i] != 2) return false;
    key = (uint32_t)c.dist[i];
  }
  return true;
}

// One radix-select pass: counts of the candidates' digit at `shift` among
// keys whose higher digits match the prefix so far, in 16 bank-staggered LDS
// copies (lane l adds to copy l % 16; see k_hist), then one global add per
// digit and block.
// The state of a select after the pick of a finished pass: the digit d at
// `shift` whose count range holds the wanted rank (counts of smaller digits
// before it), taken by every block of the next pass from that pass's counts
// (256 threads, one digit each), so that no launch is needed for the pick.
// Block 0 writes the state to `out` for the passes after.
__device__ __forceinline__ RadixSel rs_after_pick(const RadixSel* in, const uint32_t* hist, int shift, RadixSel* out) {
  __shared__ uint32_t wtot[kBlock / 64];
  __shared__ int sel_d;
  __shared__ long long sel_below;
  const RadixSel r = *in;
  if (threadIdx.x == 0) sel_d = -1;
  const int d = threadIdx.x;
  const uint32_t v = hist[d];
  uint32_t total = 0u;
  const long long before = r.below + (long long)block_scan_excl<kBlock / 64>(v, wtot, total);   // (its barriers order sel_d)
  if (r.need > 0 && before < r.need && r.need <= before + (long long)v) { sel_d = d; sel_below = before; }
  __syncthreads();
  RadixSel o = r;
  if (sel_d >= 0) {
    o.prefix |= (unsigned long long)sel_d << shift;
    o.below = sel_below;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *out = o;
  return o;
}

// The select's state for a counting pass: `in` itself for the first pass
// (in_hist null), else `in` after the pick of the previous pass's counts.
__device__ __forceinline__ RadixSel rs_state(const RadixSel* in, const uint32_t* in_hist, int in_shift,
                                             RadixSel* out) {
  return in_hist ? rs_after_pick(in, in_hist, in_shift, out) : *in;
}

template <int SEL>
__global__ __launch_bounds__(kBlock) void k_rs_hist(ScanCtx c, const RadixSel* in, const uint32_t* in_hist,
                                                    int in_shift, RadixSel* out, int shift, uint32_t* hist) {
  __shared__ uint32_t h[kHistCopies][257];
  const RadixSel rs = rs_state(in, in_hist, in_shift, out);
  for (int i = threadIdx.x; i < kHistCopies * 257; i += blockDim.x) (&h[0][0])[i] = 0u;
  __syncthreads();
  uint32_t* mine = h[threadIdx.x & (kHistCopies - 1)];
  const unsigned long long pre = rs.prefix;
  const int hi = shift + 8;   // digits above this one must match the prefix
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  auto count = [&](int64_t i) {
    unsigned long long key = 0;
    bool cand = rs_key<SEL>(c, i, key);
    if (cand && hi < 64 && (key >> hi) != (pre >> hi)) cand = false;
    if (cand) atomicAdd(&mine[(uint32_t)((key >> shift) & 0xFF)], 1u);
  };
  // four pixels per thread and step, their classes in one word (the grid is
  // small, so each thread needs several loads in flight), then the tail
  const int64_t nq = c.N >> 2;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += stride) {
    const uint32_t k4 = ((const uint32_t*)c.cls)[q];   // 4-byte aligned: in the 256-byte aligned workspace
    // classes 0, 1, 2: bit 0 marks class 1, bit 1 class 2
    if (!(k4 & (SEL == 1 ? 0x01010101u : 0x02020202u))) continue;
    // the quad's keys: (kept) four parents then four sizes, each group
    // loaded together; (other) four distances in one load
    uint32_t key[4];
    if constexpr (SEL == 1) {
      const int4 p = ((const int4*)c.parent)[q];
      const int32_t r[4] = {p.x, p.y, p.z, p.w};
#pragma unroll
      for (int b = 0; b < 4; ++b) key[b] = ~(uint32_t)c.size[r[b] < 0 ? 0 : r[b]];
    } else {
      const int4 d = ((const int4*)c.dist)[q];
      key[0] = (uint32_t)d.x; key[1] = (uint32_t)d.y; key[2] = (uint32_t)d.z; key[3] = (uint32_t)d.w;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (((k4 >> (8 * b)) & 0xFFu) != (SEL == 1 ? 1u : 2u)) continue;
      if (hi < 64 && ((unsigned long long)key[b] >> hi) != (pre >> hi)) continue;
      atomicAdd(&mine[(key[b] >> shift) & 0xFFu], 1u);
    }
  }
  if (blockIdx.x == 0)
    for (int64_t i = (nq << 2) + threadIdx.x; i < c.N; i += blockDim.x) count(i);
  __syncthreads();
  uint32_t t = 0;
  for (int k = 0; k < kHistCopies; ++k) t += h[k][threadIdx.x];
  if (t) atomicAdd(&hist[threadIdx.x], t);
}

// The pick of a select's last pass: the final state to `out` (may be `in`).
__global__ __launch_bounds__(256) void k_rs_pick(const RadixSel* in, const uint32_t* hist, int shift, RadixSel* out) {
  rs_after_pick(in, hist, shift, out);
}

// The candidates of the hash select (other pixels at the selected distance),
// compacted once, so that its eight passes read a short list instead of the
// class and distance of every pixel. Order in the list does not matter: the
// select only counts keys, and the final list comes from the raster-order
// scan. Each block takes kCandPer pixels a step, each thread four adjacent
// ones per load (a word of classes, 16 bytes of distances), and reserves
// their places with one atomic (a few hundred per image: adds to one word
// queue up one after another at the memory side).
constexpr int kCandPer = 16384;
__global__ __launch_bounds__(kBlock) void k_fc_cands(ScanCtx c, int32_t* cand, unsigned long long* ncand) {
  constexpr int kQuads = kCandPer / (4 * kBlock);   // quads per thread and step
  static_assert(kQuads * 4 * kBlock == kCandPer && 4 * kQuads <= 64, "one mask word per thread");
  __shared__ uint32_t wtot[kBlock / 64];
  __shared__ unsigned long long base;
  const FracState* f = c.fc;
  if (f->mode != 2) return;
  const int32_t dsel = (int32_t)f->s2.prefix;
  const int64_t nq = c.N >> 2;
  const uint32_t* cw = (const uint32_t*)c.cls;   // 256-byte aligned workspace arrays
  const int4* dq = (const int4*)c.dist;
  for (int64_t b0 = (int64_t)blockIdx.x * kCandPer; b0 < c.N; b0 += (int64_t)gridDim.x * kCandPer) {
    uint64_t m = 0u;   // bit 4k + b: pixel 4 (q0 + k kBlock) + b is a candidate
    const int64_t q0 = (b0 >> 2) + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kQuads; ++k) {
      const int64_t q = q0 + (int64_t)k * kBlock;
      if (q < nq) {
        const uint32_t k4 = cw[q];
        if (k4 & 0x02020202u) {   // some class-2 pixel among the four
          const int4 d = dq[q];
          const int32_t dv[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (((k4 >> (8 * b)) & 0xFFu) == 2u && dv[b] == dsel) m |= 1ull << (4 * k + b);
        }
      } else if (q == nq) {   // the last N % 4 pixels
        for (int64_t i = q << 2; i < c.N; ++i)
          if (c.cls[i] == 2 && c.dist[i] == dsel) m |= 1ull << (4 * k + (int)(i - (q << 2)));
      }
    }
    const uint32_t cnt = (uint32_t)__builtin_popcountll(m);
    uint32_t total = 0u;
    const uint32_t before = block_scan_excl<kBlock / 64>(cnt, wtot, total);
    if (threadIdx.x == 0) base = total ? atomicAdd(ncand, (unsigned long long)total) : 0ull;
    __syncthreads();
    unsigned long long pos = base + before;
    for (int k = 0; k < kQuads; ++k)
      for (int b = 0; b < 4; ++b)
        if (m >> (4 * k + b) & 1ull) cand[pos++] = (int32_t)(((q0 + (int64_t)k * kBlock) << 2) + b);
    __syncthreads();   // base is rewritten by the next step
  }
}

// One hash-select pass over the compacted candidates (as k_rs_hist).
__global__ __launch_bounds__(kBlock) void k_rs_hist_cands(const int32_t* cand, const unsigned long long* ncand,
                                                          unsigned long long seed, const RadixSel* in,
                                                          const uint32_t* in_hist, int in_shift, RadixSel* out,
                                                          int shift, uint32_t* hist) {
  __shared__ uint32_t h[kHistCopies][257];
  const RadixSel rs = rs_state(in, in_hist, in_shift, out);
  for (int i = threadIdx.x; i < kHistCopies * 257; i += blockDim.x) (&h[0][0])[i] = 0u;
  __syncthreads();
  uint32_t* mine = h[threadIdx.x & (kHistCopies - 1)];
  const unsigned long long pre = rs.prefix;
  const int hi = shift + 8;
  const int64_t n = (int64_t)*ncand;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  auto count = [&](int32_t px) {
    const unsigned long long key = mix64((unsigned long long)px ^ seed);
    if (hi < 64 && (key >> hi) != (pre >> hi)) return;
    atomicAdd(&mine[(uint32_t)((key >> shift) & 0xFF)], 1u);
  };
  // four candidates per 16-byte load (the list starts 256-byte aligned in
  // the workspace), so few threads still keep several loads in flight
  const int64_t nq = n >> 2;
  const int4* cq = (const int4*)cand;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += stride) {
    const int4 v = cq[q];
    count(v.x); count(v.y); count(v.z); count(v.w);
  }
  if (blockIdx.x == 0)
    for (int64_t k = (nq << 2) + threadIdx.x; k < n; k += blockDim.x) count(cand[k]);
  __syncthreads();
  uint32_t t = 0;
  for (int k = 0; k < kHistCopies; ++k) t += h[k][threadIdx.x];
  if (t) atomicAdd(&hist[threadIdx.x], t);
}

// Chessboard distance to the border columns and kept pixels: per column the
// vertical distance to the nearest such pixel, then per pixel the minimum
// over columns x' of max(|x - x'|, that distance), searched outwards until
// |x - x'| reaches the best found (the border columns bound it).
constexpr int32_t kFar = 1 << 30;
constexpr int kSegRows = 32;   // rows per column segment

__device__ __forceinline__ bool in_set(const ScanCtx& c, int64_t i) { return c.cls[i] != 2; }

// Per (column, 32-row segment): the last and first selected row in it.
__global__ __launch_bounds__(kBlock) void k_dt_seg(ScanCtx c, int32_t H, int32_t nseg, int32_t* last, int32_t* first) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nseg * c.W) return;
  const int x = (int)((uint32_t)t % (uint32_t)c.W), sg = (int)((uint32_t)t / (uint32_t)c.W);   // t < N < 2^31
  int lo = -1, fi = kFar;
  for (int y = sg * kSegRows; y < min(H, (sg + 1) * kSegRows); ++y)
    if (in_set(c, (int64_t)y * c.W + x)) { lo = y; if (fi == kFar) fi = y; }
  last[t] = lo;
  first[t] = fi;
}

// Per column: the nearest selected row above each segment and below it. The
// records are read kCarryBatch at a time before any result is written, so a
// thread has that many loads in flight instead of one round trip per segment.
constexpr int kCarryBatch = 16;
__global__ __launch_bounds__(kBlock) void k_dt_carry(int32_t W, int32_t nseg, const int32_t* __restrict__ last,
                                                     const int32_t* __restrict__ first, int32_t* __restrict__ up,
                                                     int32_t* __restrict__ down) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= W) return;
  int u = -kFar;
  for (int s0 = 0; s0 < nseg; s0 += kCarryBatch) {
    int v[kCarryBatch];
#pragma unroll
    for (int k = 0; k < kCarryBatch; ++k) v[k] = s0 + k < nseg ? last[(int64_t)(s0 + k) * W + x] : -1;
#pragma unroll
    for (int k = 0; k < kCarryBatch; ++k) {
      if (s0 + k >= nseg) break;
      up[(int64_t)(s0 + k) * W + x] = u;
      if (v[k] >= 0) u = v[k];
    }
  }
  int d = kFar;
  for (int s1 = nseg - 1; s1 >= 0; s1 -= kCarryBatch) {   // segments s1, s1 - 1, ...
    int v[kCarryBatch];
#pragma unroll
    for (int k = 0; k < kCarryBatch; ++k) v[k] = s1 - k >= 0 ? first[(int64_t)(s1 - k) * W + x] : kFar;
#pragma unroll
    for (int k = 0; k < kCarryBatch; ++k) {
      if (s1 - k < 0) break;
      down[(int64_t)(s1 - k) * W + x] = d;
      if (v[k] < kFar) d = v[k];
    }
  }
}

// g = vertical distance to the nearest selected pixel of the column. The
// segment's selection bits are read first (all loads in flight at once),
// then both passes run on registers and the results are written once.
__global__ __launch_bounds__(kBlock) void k_dt_col(ScanCtx c, int32_t H, int32_t nseg, const int32_t* up,
                                                   const int32_t* down, int32_t* g) {
  static_assert(kSegRows <= 32, "one mask word per segment");
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nseg * c.W) return;
  const int x = (int)((uint32_t)t % (uint32_t)c.W), sg = (int)((uint32_t)t / (uint32_t)c.W);   // t < N < 2^31
  const int y0 = sg * kSegRows, n = min(H - y0, kSegRows);
  uint32_t sel = 0u;   // bit k: row y0 + k is selected
#pragma unroll
  for (int k = 0; k < kSegRows; ++k)
    if (k < n && in_set(c, (int64_t)(y0 + k) * c.W + x)) sel |= 1u << k;
  int gv[kSegRows];
  int u = up[t];
#pragma unroll
  for (int k = 0; k < kSegRows; ++k) {
    if (sel >> k & 1u) u = y0 + k;
    gv[k] = u < 0 ? kFar : y0 + k - u;
  }
  int d = down[t];
#pragma unroll
  for (int k = kSegRows - 1; k >= 0; --k) {
    if (sel >> k & 1u) d = y0 + k;
    if (d < kFar) gv[k] = min(gv[k], d - (y0 + k));
  }
#pragma unroll
  for (int k = 0; k < kSegRows; ++k)
    if (k < n) g[(int64_t)(y0 + k) * c.W + x] = gv[k];
}

// One block per row; rows up to kRowLds pixels wide are searched in LDS,
// with the minimum of every 16 consecutive entries beside them: the search
// outwards from x skips a whole 16-entry block when even its nearest
// position and its smallest entry cannot beat the best found
// (max(|x - x'|, g(x')) >= max(distance to the block, block minimum)), so a
// pixel far from the selected set costs about d/16 + 32 steps, not d.
constexpr int kRowLds = 8192;
constexpr int kDtBlk = 16;
__global__ __launch_bounds__(kBlock) void k_dt_row(ScanCtx c, int32_t H, const int32_t* g, int32_t* dist) {
  __shared__ int32_t row[kRowLds];
  __shared__ int32_t bmin[kRowLds / kDtBlk];
  const int W = c.W;
  const bool in_lds = W <= kRowLds;
  const int nb = (W + kDtBlk - 1) / kDtBlk;
  for (int y = blockIdx.x; y < H; y += gridDim.x) {
    const int32_t* grow = g + (int64_t)y * W;
    if (in_lds) {
      for (int x = threadIdx.x; x < W; x += blockDim.x) row[x] = grow[x];
      __syncthreads();
      for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        int m = kFar;
        for (int x = b * kDtBlk; x < min(W, (b + 1) * kDtBlk); ++x) m = min(m, row[x]);
        bmin[b] = m;
      }
      __syncthreads();
      for (int x = threadIdx.x; x < W; x += blockDim.x) {
        int d = row[x];
        // right of x, then left of x; a block is skipped when its nearest
        // position is at least d away or its minimum is at least d
        for (int p = x + 1; p < W && p - x < d;) {
          const int b = p / kDtBlk;
          if (bmin[b] >= d) { p = (b + 1) * kDtBlk; continue; }
          d = min(d, max(p - x, row[p]));
          ++p;
        }
        for (int p = x - 1; p >= 0 && x - p < d;) {
          const int b = p / kDtBlk;
          if (bmin[b] >= d) { p = b * kDtBlk - 1; continue; }
          d = min(d, max(x - p, row[p]));
          --p;
        }
        dist[(int64_t)y * W + x] = d;
      }
    } else {
      for (int x = threadIdx.x; x < W; x += blockDim.x) {
        int d = grow[x];
        for (int k = 1; k < d; ++k) {
          if (x - k >= 0) d = min(d, max(k, grow[x - k]));
          if (x + k < W) d = min(d, max(k, grow[x + k]));
        }
        dist[(int64_t)y * W + x] = d;
      }
    }
    __syncthreads();
  }
}

// The same row pass for rows up to 4096 pixels (and columns up to 65535
// rows, so that g fits 16 bits), without a search per pixel. For k >= 0,
// d(x) <= k exactly when some x' with |x - x'| <= k has g(x') <= k, i.e. when
// the minimum of g over [x - k, x + k] (cut to the row) is at most k. A sparse
// table of minima over power-of-two ranges gives that minimum with two LDS
// reads. Each thread takes a run of adjacent pixels: the first by binary
// search over k, each next one from its left neighbour, since d changes by
// at most 1 from a pixel to the next (a minimum of functions of slope at most
// 1), which leaves at most two tests: k = d - 1, then k = d.
// The same pass counts the distances of the other pixels (class 2), whose
// select then needs one pick over the counts (k_fc_dist_pick) instead of
// radix passes over every pixel: distances are below W (the border columns
// are selected), so the counts have at most 4096 bins.
constexpr int kStW = 4096;
constexpr int kStLevels = 13;   // ranges of 1 .. 4096
constexpr int kStBlock = 1024;
__global__ __launch_bounds__(kStBlock) void k_dt_row_st(int32_t W, int32_t H, const int32_t* g, int32_t* dist,
                                                        const uint8_t* cls, uint32_t* dhist) {
  __shared__ uint16_t st[kStLevels][kStW];
  __shared__ uint32_t hloc[kStW];
  for (int b = threadIdx.x; b < kStW; b += kStBlock) hloc[b] = 0u;
  const int levels = 32 - __builtin_clz((unsigned)W);   // 2^(levels-1) <= W
  const int run = (W + kStBlock - 1) / kStBlock;
  // the next row's column distances are loaded while this row is searched
  constexpr int kPer = kStW / kStBlock;
  int32_t nxt[kPer];
  auto fetch = [&](int yy) {
    const int32_t* grow = g + (int64_t)yy * W;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int x = threadIdx.x + k * kStBlock;
      nxt[k] = x < W ? grow[x] : 0;
    }
  };
  if ((int)blockIdx.x < H) fetch(blockIdx.x);
  for (int y = blockIdx.x; y < H; y += gridDim.x) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int x = threadIdx.x + k * kStBlock;
      if (x < W) st[0][x] = (uint16_t)min(nxt[k], 65535);
    }
    __syncthreads();
    for (int j = 1; j < levels; ++j) {
      const int h = 1 << (j - 1);
      for (int x = threadIdx.x; x + 2 * h <= W; x += kStBlock) st[j][x] = min(st[j - 1][x], st[j - 1][x + h]);
      __syncthreads();
    }
    if (y + (int)gridDim.x < H) fetch(y + gridDim.x);
    // minimum of g over [l, r], 0 <= l <= r < W
    auto rmq = [&](int l, int r) -> int {
      const int j = 31 - __builtin_clz((unsigned)(r - l + 1));
      return (int)min(st[j][l], st[j][r - (1 << j) + 1]);
    };
    // d(x) <= k
    auto within = [&](int x, int k) -> bool { return rmq(max(0, x - k), min(W - 1, x + k)) <= k; };
    const int rowmin = rmq(0, W - 1);
    const int x0 = threadIdx.x * run, x1 = min(W, x0 + run);
    int32_t* drow = dist + (int64_t)y * W;
    if (rowmin == 65535) {
      // no selected pixel in any column of the image
      for (int x = x0; x < x1; ++x) drow[x] = kFar;
    } else if (x0 < x1) {
      // d(x0) lies in [0, hi]: the pixel's own column bounds it, and so does
      // the column holding the row minimum
      const int gx = st[0][x0];
      int lo = 0, hi = min(gx == 65535 ? kFar : gx, max(W - 1, rowmin));
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (within(x0, mid)) hi = mid;
        else lo = mid + 1;
      }
      const uint8_t* crow = cls + (int64_t)y * W;
      int d = lo;
      drow[x0] = d;
      if (crow[x0] == 2) atomicAdd(&hloc[d], 1u);
      for (int x = x0 + 1; x < x1; ++x) {
        if (d > 0 && within(x, d - 1)) d = d - 1;
        else if (!within(x, d)) d = d + 1;
        drow[x] = d;
        if (crow[x] == 2) atomicAdd(&hloc[d], 1u);
      }
    }
    __syncthreads();
  }
  for (int b = threadIdx.x; b < W; b += kStBlock)
    if (hloc[b]) atomicAdd(&dhist[b], hloc[b]);
}

// The distance select from the counts of k_dt_row_st: the smallest distance
// D whose running count reaches s2.need, and the count below it (what the
// radix passes would leave in s2). One block; each thread sums four bins.
__global__ __launch_bounds__(kStBlock) void k_fc_dist_pick(FracState* f, const uint32_t* dhist, int32_t W) {
  static_assert(kStW == 4 * kStBlock, "four bins per thread");
  __shared__ uint32_t wtot[kStBlock / 64];
  const long long need = f->s2.need;
  const int b0 = threadIdx.x * 4;
  uint32_t v[4], sum = 0u;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = b0 + k < W ? dhist[b0 + k] : 0u;
    sum += v[k];
  }
  uint32_t total = 0u;
  long long before = (long long)block_scan_excl<kStBlock / 64>(sum, wtot, total);
  if (need <= 0 || !(before < need && need <= before + (long long)sum)) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (need <= before + (long long)v[k]) {
      f->s2.prefix = (unsigned long long)(b0 + k);
      f->s2.below = before;
      return;
    }
    before += v[k];
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

size_t a256(size_t v) { return (v + 255) / 256 * 256; }

struct Layout {
  size_t L8, lab, lab2, B, parent, size, cnt, bsum, bits, hist, g, dist, frank, rhist, dhist, lut, misc, end;
};

Layout layout(int32_t W, int32_t H) {
  const int64_t N = (int64_t)W * H;
  // `dist` first holds the column pass's four per-segment arrays
  const int64_t seg_words = 4LL * ((H + kSegRows - 1) / kSegRows) * W;
  Layout o{};
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t at = off; off += a256(bytes); return at; };
  o.L8 = take(N);
  o.lab = take(N);
  o.lab2 = take(N);
  o.B = take(N);
  o.parent = take((size_t)N * 4);
  o.size = take((size_t)N * 4);
  o.cnt = take(((size_t)N + 1) * 4);
  o.bsum = take(((size_t)(N + kScanPer - 1) / kScanPer + 1) * 4);
  o.bits = take((size_t)(N + kScanPer - 1) / kScanPer * (kScanPer / 8));
  o.hist = take(256 * 8);
  o.g = take((size_t)N * 4);
  o.dist = take((size_t)std::max<int64_t>(N, seg_words) * 4);
  o.frank = take((size_t)N * 4);
  o.rhist = take(256 * 4 * kRsPasses * 3);   // one zeroed count array per pass of each of the three selects
  o.dhist = take(kStW * 4);
  o.lut = take(256);
  o.misc = take(kMiscBytes);
  o.end = off;
  return o;
}

// The steps of L8(Y) for k_light: L8 = round half away from zero of
// (116 f(Y) - 16) * 255 / 100, clamped to [0, 255], with f the CIE function
// (cube root above (6/29)^3, linear below), all in fp64. For each v, a binary
// search over the ordered bit patterns of the non-negative doubles up to 2
// finds the smallest Y with L8(Y) >= v. Computed once per process.
const LightSteps& light_steps() {
  static const LightSteps steps = [] {
#pragma clang fp contract(off)
    LightSteps r{};
    const double e = 6.0 / 29.0;
    const double e3 = e * e * e, k3 = 3 * e * e;
    auto l8 = [&](double Y) -> int {
      const double f = Y > e3 ? std::cbrt(Y) : Y / k3 + 4.0 / 29.0;
      const double s = (116.0 * f - 16.0) * 255.0 / 100.0;
      const double q = s >= 0 ? std::floor(s + 0.5) : -std::floor(-s + 0.5);
      return q < 0 ? 0 : (q > 255 ? 255 : (int)q);
    };
    auto at = [](uint64_t b) { double d; std::memcpy(&d, &b, 8); return d; };
    uint64_t hi_bits;
    const double two = 2.0;
    std::memcpy(&hi_bits, &two, 8);
    r.t[0] = 0.0;
    for (int v = 1; v < 256; ++v) {
      if (l8(two) < v) { r.t[v] = HUGE_VAL; continue; }
      uint64_t lo = 0, hi = hi_bits;   // l8(at(hi)) >= v
      while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (l8(at(mid)) >= v) hi = mid; else lo = mid + 1;
      }
      r.t[v] = at(lo);
    }
    return r;
  }();
  return steps;
}

void launch_light(const uint8_t* img, int32_t W, int32_t H, int32_t C, int64_t pitch, uint8_t* L8, int grid,
                  hipStream_t s) {
  // the bucket table of k_light4 needs consecutive steps more than a bucket apart
  static const bool coarse_ok = [] {
    const LightSteps& st = light_steps();
    for (int k = 1; k < 255; ++k)
      if (std::isfinite(st.t[k + 1]) && !(st.t[k + 1] - st.t[k] > 1.0 / kLightBuckets)) return false;
    return true;
  }();
  if (C == 1)
    hipLaunchKernelGGL(k_gray, dim3(grid), dim3(kBlock), 0, s, img, W, H, pitch, L8);
  else if (coarse_ok && (W & 3) == 0 && (pitch & 3) == 0 && ((uintptr_t)img & 3) == 0 && ((uintptr_t)L8 & 3) == 0)
    hipLaunchKernelGGL(k_light4, dim3(std::min(grid, 1024)), dim3(kBlock), 0, s, img, W, H, pitch, L8,
                       light_steps());
  else
    hipLaunchKernelGGL(k_light, dim3(grid), dim3(kBlock), 0, s, img, W, H, C, pitch, L8, light_steps());
}

int grid_for(int64_t n) {
  const int64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

}  // namespace sbs_front

using namespace sbs_front;

extern "C" {

int sbs_lightness(const uint8_t* img, int32_t W, int32_t H, int32_t C, int64_t pitch, uint8_t* out_l8, void* stream) {
  if (W < 1 || H < 1 || (int64_t)W * H > INT32_MAX || (C != 1 && C != 3) || pitch < (int64_t)W * C)
    return fail(SBS_ERR_INVALID_ARG, "bad image geometry");
  if (!img || !out_l8) return fail(SBS_ERR_INVALID_ARG, "NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  launch_light(img, W, H, C, pitch, out_l8, grid_for((int64_t)W * H), s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SBS_ERR_HIP, "lightness: %s", hipGetErrorString(e));
  return SBS_OK;
}

size_t sbs_boundaries_workspace_bytes(int32_t W, int32_t H) {
  if (W < 1 || H < 1 || (int64_t)W * H > INT32_MAX) return 0;
  return layout(W, H).end;
}

int sbs_boundaries(const uint8_t* img, int32_t W, int32_t H, int32_t C, int64_t pitch, int32_t K, int32_t mode,
                   int32_t min_cc, double frac, uint64_t seed, uint32_t* out_idx, int64_t* out_count,
                   uint8_t* out_refined, uint8_t* out_labels, void* workspace, size_t workspace_bytes, void* stream) {
  if (W < 1 || H < 1 || (int64_t)W * H > INT32_MAX || (C != 1 && C != 3) || pitch < (int64_t)W * C)
    return fail(SBS_ERR_INVALID_ARG, "bad image geometry");
  if (!img || !out_idx || !out_count || !workspace) return fail(SBS_ERR_INVALID_ARG, "NULL pointer");
  if (K < 1 || K > kMaxK) return fail(SBS_ERR_INVALID_ARG, "K must be in [1, %d]", kMaxK);
  if (mode != 0 && mode != 1) return fail(SBS_ERR_INVALID_ARG, "mode must be 0 (configured) or 1 (paper)");
  if (mode == 0 && min_cc < 0) return fail(SBS_ERR_INVALID_ARG, "min_cc < 0");
  if (H > 4 * 65535) return fail(SBS_ERR_UNSUPPORTED, "H > %d", 4 * 65535);   // 2-D stencil grid: 4 rows per block
  if (!(frac < 0.0) && !(frac <= 1.0)) return fail(SBS_ERR_INVALID_ARG, "frac must be < 0 (off) or in [0, 1]");
  const int64_t N = (int64_t)W * H;
  const Layout Lo = layout(W, H);
  if (workspace_bytes < Lo.end) return fail(SBS_ERR_INVALID_ARG, "workspace too small");
  if ((uintptr_t)workspace & 255) return fail(SBS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)workspace;
  uint8_t* L8 = (uint8_t*)(base + Lo.L8);
  uint8_t* lab = (uint8_t*)(base + Lo.lab);
  uint8_t* lab2 = (uint8_t*)(base + Lo.lab2);
  uint8_t* B = (uint8_t*)(base + Lo.B);
  int32_t* parent = (int32_t*)(base + Lo.parent);
  int32_t* size = (int32_t*)(base + Lo.size);
  int32_t* cnt = (int32_t*)(base + Lo.cnt);
  uint32_t* bsum = (uint32_t*)(base + Lo.bsum);
  unsigned long long* hist = (unsigned long long*)(base + Lo.hist);
  uint8_t* lut = (uint8_t*)(base + Lo.lut);
  char* misc = base + Lo.misc;
  int32_t* passes = (int32_t*)misc;
  unsigned long long* total = (unsigned long long*)(misc + 128);
  DropRule* rule = (DropRule*)(misc + 192);
  FracState* fs = (FracState*)(misc + 256);
  unsigned long long* n1 = (unsigned long long*)(misc + 1024);   // kN1Parts partial counts
  RadixSel* rsv = (RadixSel*)(misc + 704);   // a select's state after each pass's pick (kRsPasses)
  static_assert(704 + kRsPasses * sizeof(RadixSel) <= 1024, "misc layout");
  int32_t* gcol = (int32_t*)(base + Lo.g);
  int32_t* dist = (int32_t*)(base + Lo.dist);
  int32_t* frank = (int32_t*)(base + Lo.frank);
  uint32_t* rhist = (uint32_t*)(base + Lo.rhist);
  static_assert(sizeof(FracState) <= 256, "misc layout");
  const int g = grid_for(N);

  // Clear the small counters with kernels (no memset nodes if the caller captures the stream).
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(kBlock), 0, s, (uint8_t*)hist, (int64_t)(256 * 8), (uint8_t)0);
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(kBlock), 0, s, (uint8_t*)misc, (int64_t)kMiscBytes, (uint8_t)0);
  // grey rows without gaps are the lightness image itself (no copy)
  const uint8_t* lum = L8;
  if (C == 1 && pitch == W) lum = img;
  else launch_light(img, W, H, C, pitch, L8, g, s);
  // at most 512 blocks: each ends with up to 256 global adds
  hipLaunchKernelGGL(k_hist, dim3(std::min(grid_for((N + 15) / 16), 512)), dim3(kBlock), 0, s, lum, N, hist);
  hipLaunchKernelGGL(k_kmeans, dim3(1), dim3(256), 0, s, hist, K, lut, passes);
  hipLaunchKernelGGL(k_label, dim3(g), dim3(kBlock), 0, s, lum, N, lut, lab);
  const uint8_t* labels = lab;
  if (mode == 0) {
    // open, close and boundary in one pass; the closed labels go straight to
    // out_labels when asked for
    const dim3 gm((W + kMorphT - 1) / kMorphT, (H + kMorphT - 1) / kMorphT);
    // word-wide interior path: rows of whole words, the outputs word-aligned too
    const int32_t words = (W & 3) == 0 && ((uintptr_t)out_labels & 3) == 0 ? 1 : 0;
    hipLaunchKernelGGL(k_morph_refine, gm, dim3(kBlock), 0, s, lab, W, H, B, out_labels, words);
    labels = nullptr;
  } else {
    // boundary, fill and remove in one pass
    const dim3 gm((W + kMorphT - 1) / kMorphT, (H + kMorphT - 1) / kMorphT);
    hipLaunchKernelGGL(k_paper_refine, gm, dim3(kBlock), 0, s, lab, W, H, B, (W & 3) == 0 ? 1 : 0);
  }
  if (out_labels && labels) {
    const hipError_t ce = hipMemcpyAsync(out_labels, labels, (size_t)N, hipMemcpyDeviceToDevice, s);
    if (ce != hipSuccess) return fail(SBS_ERR_HIP, "boundaries: %s", hipGetErrorString(ce));
  }
  const dim3 gt((W + kTileW - 1) / kTileW, (H + kTileH - 1) / kTileH);
  hipLaunchKernelGGL(k_cc_tile, gt, dim3(kBlock), 0, s, B, W, H, parent, size);
  hipLaunchKernelGGL(k_cc_edges, gt, dim3(128), 0, s, B, W, H, parent);
  hipLaunchKernelGGL(k_cc_flatten, dim3(g), dim3(kBlock), 0, s, N, parent, size);

  const int64_t nb = (N + kScanPer - 1) / kScanPer;
  ScanCtx c{};
  c.B = B; c.parent = parent; c.size = size; c.rule = nullptr; c.min_cc = min_cc; c.W = W; c.N = N;
  c.rank = cnt;   // the rank array reuses cnt: ranks are written after k_drop_find has read the counts
  c.out = out_idx; c.refined = out_refined; c.count = (long long*)out_count;
  c.bits = (unsigned long long*)(base + Lo.bits);
  if (mode == 1) {
    hipLaunchKernelGGL(k_fill, dim3(g), dim3(kBlock), 0, s, (uint8_t*)cnt, (int64_t)(N + 1) * 4, (uint8_t)0);
    // at most 512 blocks: each block's closing adds (its total and its small
    // sizes' counts) go to the same few global words, so fewer blocks wait less
    hipLaunchKernelGGL(k_drop_count, dim3(std::min(g, 512)), dim3(kBlock), 0, s, size, N, total, cnt);
    hipLaunchKernelGGL(k_drop_find, dim3(1), dim3(1024), 0, s, cnt, total, 0.04, rule);
    c.rule = rule;
    // rank of each root of size s* among those roots, in raster order
    hipLaunchKernelGGL(k_scan_count<0>, dim3((unsigned)nb), dim3(kBlock), 0, s, c, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, nb, (long long*)nullptr);
    hipLaunchKernelGGL(k_scan_apply<0>, dim3((unsigned)nb), dim3(kBlock), 0, s, c, bsum);
  }
  if (frac >= 0.0) {
    const long long want = std::min<long long>((long long)N, std::llround(frac * (double)N));
    const long long n0 = W == 1 ? H : 2LL * H;
    uint8_t* cls = lab2;   // free once the refinement is done
    hipLaunchKernelGGL(k_fc_class, dim3(g), dim3(kBlock), 0, s, c, cls, n1);
    // Component sizes are at most N: with N below 2^24 the top digit of ~size is
    // 0xFF for every kept pixel, so it is set here and its pass skipped.
    const bool small = N < (1LL << 24);
    hipLaunchKernelGGL(k_fc_plan, dim3(1), dim3(1), 0, s, fs, n1, want, n0, small ? 0xFF000000ull : 0ull);
    c.fc = fs; c.dist = dist; c.frank = frank; c.seed = (unsigned long long)seed; c.cls = cls;
    // radix-select histograms: at most 512 blocks (each ends with up to 256
    // global adds). Pass p counts into its own zeroed array and starts from
    // the state after the pick of pass p - 1's counts (rsv[p - 1], written by
    // its block 0); one pick launch after the last pass sets the final state.
    const int gr = std::min(g, 512);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(kBlock), 0, s, (uint8_t*)rhist, (int64_t)(256 * 4 * kRsPasses * 3),
                       (uint8_t)0);
    int nsel = 0;
    auto select = [&](RadixSel* st, int first_shift, int last_shift, auto launch_pass) {
      uint32_t* const hs = rhist + 256 * kRsPasses * nsel++;   // this select's count arrays
      int p = 0, prev_shift = 0;
      for (int sh = first_shift; sh >= last_shift; sh -= 8, ++p) {
        const RadixSel* in = p <= 1 ? st : &rsv[p - 1];
        const uint32_t* in_hist = p == 0 ? nullptr : hs + 256 * (p - 1);
        launch_pass(in, in_hist, prev_shift, &rsv[p], sh, hs + 256 * p);
        prev_shift = sh;
      }
      hipLaunchKernelGGL(k_rs_pick, dim3(1), dim3(256), 0, s, p <= 1 ? (const RadixSel*)st : &rsv[p - 1],
                         hs + 256 * (p - 1), prev_shift, st);
    };
    select(&fs->s1, small ? 16 : 24, 0,   // kept pixels: size descending
           [&](const RadixSel* in, const uint32_t* ih, int ish, RadixSel* out, int sh, uint32_t* h) {
             hipLaunchKernelGGL(k_rs_hist<1>, dim3(gr), dim3(kBlock), 0, s, c, in, ih, ish, out, sh, h);
           });
    hipLaunchKernelGGL(k_scan_count<2>, dim3((unsigned)nb), dim3(kBlock), 0, s, c, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, nb, (long long*)nullptr);
    hipLaunchKernelGGL(k_scan_apply<2>, dim3((unsigned)nb), dim3(kBlock), 0, s, c, bsum);
    {
      // segment summaries live in `dist` until the column pass is done
      const int nseg = (H + kSegRows - 1) / kSegRows;
      const int64_t ns = (int64_t)nseg * W;
      int32_t* last = dist;
      int32_t* first = dist + ns;
      int32_t* up = dist + 2 * ns;
      int32_t* down = dist + 3 * ns;
      const unsigned gs = (unsigned)((ns + kBlock - 1) / kBlock);
      hipLaunchKernelGGL(k_dt_seg, dim3(gs), dim3(kBlock), 0, s, c, H, nseg, last, first);
      hipLaunchKernelGGL(k_dt_carry, dim3((W + kBlock - 1) / kBlock), dim3(kBlock), 0, s, W, nseg, last, first, up, down);
      hipLaunchKernelGGL(k_dt_col, dim3(gs), dim3(kBlock), 0, s, c, H, nseg, up, down, gcol);
    }
    if (W <= kStW && H <= 65535) {
      // one block per CU (the table takes most of the LDS), each over rows in turn
      uint32_t* dhist = (uint32_t*)(base + Lo.dhist);
      hipLaunchKernelGGL(k_fill, dim3(1), dim3(kBlock), 0, s, (uint8_t*)dhist, (int64_t)(kStW * 4), (uint8_t)0);
      hipLaunchKernelGGL(k_dt_row_st, dim3(H < 256 ? H : 256), dim3(kStBlock), 0, s, W, H, gcol, dist, cls, dhist);
      hipLaunchKernelGGL(k_fc_dist_pick, dim3(1), dim3(kStBlock), 0, s, fs, dhist, W);
    } else {
      hipLaunchKernelGGL(k_dt_row, dim3(H < 16384 ? H : 16384), dim3(kBlock), 0, s, c, H, gcol, dist);
      // Distances are below W (the border columns are selected), so digits at
      // and above a power of two >= W are 0 for every candidate: the pick
      // would add 0 to the prefix and to the count below, so those passes are skipped.
      int top = 24;
      while (top >= 8 && (int64_t)W <= (1LL << top)) top -= 8;
      select(&fs->s2, top, 0,   // other pixels: distance
             [&](const RadixSel* in, const uint32_t* ih, int ish, RadixSel* out, int sh, uint32_t* h) {
               hipLaunchKernelGGL(k_rs_hist<2>, dim3(gr), dim3(kBlock), 0, s, c, in, ih, ish, out, sh, h);
             });
    }
    hipLaunchKernelGGL(k_fc_after_dist, dim3(1), dim3(1), 0, s, fs);
    // other pixels at that distance: hash, over their compacted list (in the
    // column-distance buffer, free once the row pass has run)
    int32_t* cand = gcol;
    unsigned long long* ncand = (unsigned long long*)(misc + 640);
    hipLaunchKernelGGL(k_fc_cands, dim3((unsigned)std::min<int64_t>((N + kCandPer - 1) / kCandPer, 8192)),
                       dim3(kBlock), 0, s, c, cand, ncand);
    select(&fs->s3, 56, 0,   // the hash
           [&](const RadixSel* in, const uint32_t* ih, int ish, RadixSel* out, int sh, uint32_t* h) {
             hipLaunchKernelGGL(k_rs_hist_cands, dim3(std::min(gr, 64)), dim3(kBlock), 0, s, cand, ncand,
                                (unsigned long long)seed, in, ih, ish, out, sh, h);
           });
    hipLaunchKernelGGL(k_scan_count<3>, dim3((unsigned)nb), dim3(kBlock), 0, s, c, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, nb, (long long*)nullptr);
    hipLaunchKernelGGL(k_scan_apply<3>, dim3((unsigned)nb), dim3(kBlock), 0, s, c, bsum);
  }
  // the kept map, when asked for, is worked out per element in the applying
  // pass anyway: the flags are then worked out there too
  if (out_refined) c.bits = nullptr;
  hipLaunchKernelGGL(k_scan_count<1>, dim3((unsigned)nb), dim3(kBlock), 0, s, c, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, nb, (long long*)out_count);
  hipLaunchKernelGGL(k_scan_apply<1>, dim3((unsigned)nb), dim3(kBlock), 0, s, c, bsum);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SBS_ERR_HIP, "boundaries: %s", hipGetErrorString(e));
  return SBS_OK;
}

}  // extern "C"
