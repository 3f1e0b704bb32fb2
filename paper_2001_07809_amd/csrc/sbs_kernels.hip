// HIP kernels for boundary-pixel SAD-WTA on gfx950.
//
// The operation (arXiv 2001.07809, Sec. III "Disparity Measurement of Boundary
// Pixels"; winner-takes-all, Sec. II): for each listed pixel, the disparity d
// in [0, dmax] that minimises the w x w (x channels) sum of absolute
// differences between the left window at x and the right window at x - d on
// the same rows, with replicate padding and ties to the smaller d.
//
// Tiled path (per frame):
//   k_prep      replicate-padded RGBx copies of both images (one u32 per pixel,
//               so one v_sad_u8 covers all channels of a pixel) and a cleared
//               pixel->slot map.
//   k_scatter   map[p] = largest list slot k with idx[k] == p; keys[k] = max.
//   k_rowbits   per image row, one bit per 64-column group holding a listed pixel.
//   k_tile_*    the column-sum kernel. One wavefront owns a tile of output
//               columns x rows and a chunk of disparities. Each lane owns four
//               adjacent window columns. Walking down the tile's rows it keeps,
//               per (column, disparity), running sums of the absolute
//               differences entering and leaving the w-row window (two
//               v_sad_u8 per column, disparity and row). On a row that holds
//               listed pixels it forms prefix sums along the row (in-lane, then
//               a DPP scan across lanes), stores them in LDS, and each listed
//               pixel reads its window sum as a difference of two prefix
//               entries, then folds (cost << 8 | d) into its slot's key with an
//               atomic minimum.
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

// ---------------------------------------------------------------------------
// Descriptor upload: the descriptors travel inside the kernel argument, so a
// captured graph replays them without touching host memory.
__global__ void k_put_desc(FrameDev* table, DescBatch b) {
  int i = threadIdx.x;
  if (i < b.count) table[b.first + i] = b.f[i];
}

__global__ void k_reset_head(WsHeader* h) {
  if (threadIdx.x == 0) h->head = 0ull;
}

// Padded copies and map clearing. grid: (blocks, frames); frames offset by f0.
__global__ __launch_bounds__(256) void k_prep(const FrameDev* __restrict__ table, int f0) {
  const FrameDev& f = table[f0 + blockIdx.y];
  const int W = f.W, H = f.H, C = f.C, r = f.r;
  for (int v = blockIdx.x; v < f.ph; v += gridDim.x) {
    const int y = clampi(v - r, 0, H - 1);
    const uint8_t* lrow = f.left + (int64_t)y * f.pitch;
    const uint8_t* rrow = f.right + (int64_t)y * f.pitch;
    uint32_t* lo = f.lp + (int64_t)v * f.lpw;
    uint32_t* ro = f.rp + (int64_t)v * f.rpw;
    for (int u = threadIdx.x; u < f.lpw; u += blockDim.x) lo[u] = load_px(lrow, clampi(u - r, 0, W - 1), C);
    for (int u = threadIdx.x; u < f.rpw; u += blockDim.x) ro[u] = load_px(rrow, clampi(u - r - f.roff, 0, W - 1), C);
  }
  const int64_t N = (int64_t)W * H;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    f.map[i] = -1;
}

// map[p] = max k with idx[k] == p; keys cleared; out-of-range entries answered.
__global__ __launch_bounds__(256) void k_scatter(const FrameDev* __restrict__ table, int f0, WsHeader* hdr) {
  const FrameDev& f = table[f0 + blockIdx.y];
  const int64_t N = (int64_t)f.W * f.H;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < f.n; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = f.idx[k];
    f.keys[k] = 0xFFFFFFFFu;
    if ((int64_t)p < N) {
      atomicMax(&f.map[p], (int32_t)k);
    } else {
      f.out_disp[k] = 255;
      if (f.out_cost) f.out_cost[k] = 0xFFFFFFFFu;
      atomicOr(&hdr->error, 1u);
    }
  }
}

// rowbits[y * rbw + w] bit g: some column in [64 (64 w + g), +64) of row y is listed.
// One wavefront per (row, word); grid: (ceil(H * rbw / 4), frames), 256 threads.
__global__ __launch_bounds__(256) void k_rowbits(const FrameDev* __restrict__ table, int f0) {
  const FrameDev& f = table[f0 + blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int64_t job = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (job >= (int64_t)f.H * f.rbw) return;
  const int y = (int)(job / f.rbw), w = (int)(job % f.rbw);
  const int32_t* mrow = f.map + (int64_t)y * f.W;
  uint64_t word = 0;
  for (int g = 0; g < 64; ++g) {
    const int x = (w * 64 + g) * 64 + lane;
    const bool hit = x < f.W && mrow[x] >= 0;
    if (__builtin_amdgcn_ballot_w64(hit)) word |= 1ull << g;
  }
  if (lane == 0) f.rowbits[job] = word;
}

// ---------------------------------------------------------------------------
// Wave-wide inclusive prefix sum with DPP: shifts within rows of 16 lanes,
// then broadcasts of lane 15 and lane 31 to the rows above.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

template <int DC>
struct TileLds {
  uint32_t pre[DC][kSpan];   // inclusive prefix sums of the window-column sums along the row
  int32_t eo[kSpan];         // listed pixels of the current row: output column offset
  int32_t es[kSpan];         //                                 and representative slot
};

// Global-memory views (the descriptor's pointers are generic; these let the
// compiler emit global_load instead of flat_load).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 g_uint4;
typedef __attribute__((address_space(1))) const int32_t g_int32;
typedef __attribute__((address_space(1))) const uint64_t g_uint64;

// Loads the pixels one lane needs from padded row `row`: its four left
// columns, and the DC + 3 right columns that pair with them over the chunk
// (right index c + DC - 1 - k pairs with left column c at disparity d0 + k).
template <int DC>
__device__ __forceinline__ void load_row(const FrameDev& f, int row, int lcol, int rbase, uint32_t (&L)[4],
                                         uint32_t (&R)[DC + 4]) {
  const u32x4 lv = *(g_uint4*)(f.lp + (int64_t)row * f.lpw + lcol);
  L[0] = lv.x; L[1] = lv.y; L[2] = lv.z; L[3] = lv.w;
  g_uint4* rsrc = (g_uint4*)(f.rp + (int64_t)row * f.rpw + rbase);
#pragma unroll
  for (int q = 0; q < DC / 4 + 1; ++q) {
    const u32x4 t = rsrc[q];
    R[4 * q + 0] = t.x; R[4 * q + 1] = t.y; R[4 * q + 2] = t.z; R[4 * q + 3] = t.w;
  }
}

// One work item = (tile, disparity chunk) of one frame.
template <int DC>
__device__ __forceinline__ void tile_item(const FrameDev& f, int64_t item, TileLds<DC>& sm) {
  const int lane = threadIdx.x;
  const int chunk = (int)(item % f.nch);
  const int64_t tile = item / f.nch;
  const int tx = (int)(tile % f.ntx), tyi = (int)(tile / f.ntx);
  const int W = f.W, H = f.H, r = f.r;
  const int x0 = tx * f.txo, y0 = tyi * f.ty;
  const int x1 = min(x0 + f.txo, W), y1 = min(y0 + f.ty, H);
  const int d0 = chunk * DC;
  const int dcount = min(DC, f.dmax + 1 - d0);

  // Rows of this tile holding a listed pixel in [x0, x1).
  bool act = false;
  {
    const int y = y0 + lane;
    if (lane < f.ty && y < y1) {
      const int g0 = x0 >> 6, g1 = (x1 - 1) >> 6;
      for (int w = g0 >> 6; w <= (g1 >> 6); ++w) {
        const uint64_t bits = *(g_uint64*)(f.rowbits + (int64_t)y * f.rbw + w);
        const int lo = max(g0 - 64 * w, 0), hi = min(g1 - 64 * w, 63);
        const uint64_t m = (hi == 63 ? ~0ull : ((1ull << (hi + 1)) - 1)) & ~((1ull << lo) - 1);
        if (bits & m) act = true;
      }
    }
  }
  const uint64_t rows = __builtin_amdgcn_ballot_w64(act);
  if (rows == 0) return;
  const int ya = y0 + __builtin_ctzll(rows);
  const int yb = y0 + 63 - __builtin_clzll(rows);

  const int lcol = x0 + kColsPerLane * lane;
  const int rbase = x0 + kColsPerLane * lane - d0 - (DC - 1) + f.roff;

  // cad[c][k]: sum over the window's rows of the absolute differences in
  // window column 4 lane + c at disparity d0 + k.
  uint32_t cad[kColsPerLane][DC];
#pragma unroll
  for (int c = 0; c < kColsPerLane; ++c)
#pragma unroll
    for (int k = 0; k < DC; ++k) cad[c][k] = 0;

  // Window of output row ya: padded rows ya .. ya + 2r.
  for (int row = ya; row <= ya + 2 * r; ++row) {
    uint32_t L[4], R[DC + 4];
    load_row<DC>(f, row, lcol, rbase, L, R);
#pragma unroll
    for (int c = 0; c < kColsPerLane; ++c)
#pragma unroll
      for (int k = 0; k < DC; ++k) cad[c][k] = __builtin_amdgcn_sad_u8(L[c], R[c + DC - 1 - k], cad[c][k]);
  }

  for (int y = ya; y <= yb; ++y) {
    if ((rows >> (y - y0)) & 1ull) {
      // Prefix sums of the window-column sums along the row, to LDS.
#pragma unroll
      for (int k = 0; k < DC; ++k) {
        const uint32_t q0 = cad[0][k];
        const uint32_t q1 = q0 + cad[1][k];
        const uint32_t q2 = q1 + cad[2][k];
        const uint32_t q3 = q2 + cad[3][k];
        const uint32_t excl = wave_incl_scan(q3) - q3;
        uint4 o;
        o.x = excl + q0; o.y = excl + q1; o.z = excl + q2; o.w = excl + q3;
        *reinterpret_cast<uint4*>(&sm.pre[k][kColsPerLane * lane]) = o;
      }
      // Listed pixels of this row owned by this tile (output offset o = window column - r).
      int total = 0;
#pragma unroll
      for (int c = 0; c < kColsPerLane; ++c) {
        const int o = kColsPerLane * lane + c - r;
        int32_t m = -1;
        if (o >= 0 && x0 + o < x1) m = *(g_int32*)(f.map + (int64_t)y * W + x0 + o);
        const uint64_t b = __builtin_amdgcn_ballot_w64(m >= 0);
        if (m >= 0) {
          const int pos = total + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
          sm.eo[pos] = o;
          sm.es[pos] = m;
        }
        total += __builtin_popcountll(b);
      }
      __syncthreads();
      for (int e0 = 0; e0 < total; e0 += kWave) {
        const int e = e0 + lane;
        if (e < total) {
          const int o = sm.eo[e];
          const int s = sm.es[e];
          uint32_t best = 0xFFFFFFFFu;
#pragma unroll
          for (int k = 0; k < DC; ++k) {
            if (k < dcount) {
              const uint32_t hi = sm.pre[k][o + 2 * r];
              const uint32_t lo = o > 0 ? sm.pre[k][o - 1] : 0u;
              best = min(best, ((hi - lo) << 8) | (uint32_t)(d0 + k));
            }
          }
          atomicMin(&f.keys[s], best);
        }
      }
      __syncthreads();
    }
    if (y < yb) {
      // Slide the window down one row: add padded row y + 2r + 1, drop padded row y.
      uint32_t Ln[4], Rn[DC + 4], Lo[4], Ro[DC + 4];
      load_row<DC>(f, y + 2 * r + 1, lcol, rbase, Ln, Rn);
      load_row<DC>(f, y, lcol, rbase, Lo, Ro);
#pragma unroll
      for (int c = 0; c < kColsPerLane; ++c)
#pragma unroll
        for (int k = 0; k < DC; ++k) {
          const uint32_t out = __builtin_amdgcn_sad_u8(Lo[c], Ro[c + DC - 1 - k], 0u);
          cad[c][k] = __builtin_amdgcn_sad_u8(Ln[c], Rn[c + DC - 1 - k], cad[c][k]) - out;
        }
    }
  }
}

template <int DC>
__global__ __launch_bounds__(64) void k_tile_grid(const FrameDev* __restrict__ table, int fi) {
  __shared__ TileLds<DC> sm;
  const FrameDev& f = table[fi];
  tile_item<DC>(f, (int64_t)blockIdx.x, sm);
}

// Persistent form: every workgroup pops work items of all frames from one queue.
template <int DC>
__global__ __launch_bounds__(64) void k_tile_persistent(const FrameDev* __restrict__ table, int nframes,
                                                        int64_t total, WsHeader* hdr) {
  __shared__ TileLds<DC> sm;
  __shared__ long long next_item;
  for (;;) {
    if (threadIdx.x == 0) next_item = (long long)atomicAdd(&hdr->head, 1ull);
    __syncthreads();
    const int64_t it = next_item;
    __syncthreads();
    if (it >= total) return;
    // frame of this item: last frame with item_base <= it
    int lo = 0, hi = nframes - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (table[mid].item_base <= it) lo = mid; else hi = mid - 1;
    }
    const FrameDev& f = table[lo];
    tile_item<DC>(f, it - f.item_base, sm);
  }
}

__global__ __launch_bounds__(256) void k_finalize(const FrameDev* __restrict__ table, int f0) {
  const FrameDev& f = table[f0 + blockIdx.y];
  const int64_t N = (int64_t)f.W * f.H;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < f.n; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = f.idx[k];
    if ((int64_t)p >= N) continue;
    const uint32_t key = f.keys[f.map[p]];
    f.out_disp[k] = (uint8_t)(key & 0xFFu);
    if (f.out_cost) f.out_cost[k] = key >> 8;
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

hipError_t launch_prologue(const FrameDev* table, int f0, int nf, int max_rows, int max_rbjobs, WsHeader* hdr,
                           hipStream_t s) {
  int gx = max_rows < 1024 ? max_rows : 1024;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_prep, dim3(gx, nf), dim3(256), 0, s, table, f0);
  hipLaunchKernelGGL(k_scatter, dim3(256, nf), dim3(256), 0, s, table, f0, hdr);
  int gr = (max_rbjobs + 3) / 4;
  if (gr < 1) gr = 1;
  hipLaunchKernelGGL(k_rowbits, dim3(gr, nf), dim3(256), 0, s, table, f0);
  return hipGetLastError();
}

hipError_t launch_finalize(const FrameDev* table, int f0, int nf, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(256, nf), dim3(256), 0, s, table, f0);
  return hipGetLastError();
}

hipError_t launch_tile_grid(const FrameDev* table, int fi, int64_t nitems, int chunk, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (chunk == 8) hipLaunchKernelGGL(k_tile_grid<8>, dim3((unsigned)nitems), dim3(64), 0, s, table, fi);
  else hipLaunchKernelGGL(k_tile_grid<16>, dim3((unsigned)nitems), dim3(64), 0, s, table, fi);
  return hipGetLastError();
}

hipError_t launch_tile_persistent(const FrameDev* table, int nframes, int64_t total, int chunk, int grid,
                                  WsHeader* hdr, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_head, dim3(1), dim3(64), 0, s, hdr);
  if (total <= 0) return hipGetLastError();
  if (chunk == 8)
    hipLaunchKernelGGL(k_tile_persistent<8>, dim3(grid), dim3(64), 0, s, table, nframes, total, hdr);
  else
    hipLaunchKernelGGL(k_tile_persistent<16>, dim3(grid), dim3(64), 0, s, table, nframes, total, hdr);
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
