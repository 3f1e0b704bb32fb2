// Internal definitions shared by the HIP kernels and the host layer of libsbs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sbs {

constexpr int kWave = 64;
constexpr int kMaxSpan = kWave * 8;        // window columns of a tile at 8 columns per lane (512)
constexpr int kMaxChunk = 16;         // largest disparity chunk a kernel instance handles
constexpr int kMaxTileRows = 256;     // largest tile height (four 64-bit row masks)
constexpr int kDescPerLaunch = 8;          // descriptors carried by one upload kernel
constexpr uint32_t kUnsorted = 1u;         // FrameDev::state bit
constexpr int kQueues = 8;                 // one work queue per XCD; tile t's items go to queue t % 8

// Per-frame descriptor as the kernels see it (lives in the workspace).
struct FrameDev {
  const uint8_t* left;
  const uint8_t* right;
  const uint32_t* idx;
  uint8_t* out_disp;
  uint32_t* out_cost;
  int32_t* map;        // W*H: a representative list slot per pixel, or -1
  uint32_t* keys;      // n: (cost << 8) | d, running minimum per representative slot
  uint32_t* lp;        // left copy, RGBx u32 per pixel, replicate-padded (edge bands only when linpl)
  uint32_t* rp;        // right copy, RGBx u32 per pixel, replicate-padded
  uint64_t* rowbits;   // per row: one bit per 64-column group holding a listed pixel
  uint32_t* state;     // state[0] bit 0: the list is not in strictly increasing raster order;
                       // state[2..3]: u64, the first list slot holding an index >= W*H (n if none)
  int32_t* tptr;       // sorted lists: tptr[y * tpw + t] = first list slot >= y*W + t*txo
  int64_t pitch;       // bytes between image rows
  int64_t n;           // list length
  int64_t item_base;   // first work item of this frame in the batch (one-queue order)
  int64_t nitems;      // work items of this frame (tiles x chunks)
  int64_t xbase[kQueues];  // first item of this frame in each XCD queue
  int32_t W, H, C;
  int32_t r, dmax;
  int32_t lpw, rpw, ph;  // padded copy widths (u32 units) and height (rows)
  int32_t lpad, rpad;    // copy column of image column c: c + lpad (left), c + rpad (right); multiples of 4
  int32_t rbw;           // u64 words per row in rowbits
  int32_t txo, ty;       // tile: output columns and rows
  int32_t ntx, nty;      // tiles per row / column
  int32_t nch, chunk;    // disparity chunks and their size
  int32_t tpw;           // entries per row of tptr (ntx + 1)
  int32_t pack;          // 1: the sum of two window columns (<= 2 * block * 255 * C) fits in 16 bits
  int32_t cpl;           // window columns per lane: 4, or 8 (ordered lists, 8-disparity chunks, pack == 1)
  int32_t linpl;         // 1: tiles whose window lies inside the image read the left image in place
                         // (C == 3, 4-byte-aligned rows); the left copy then holds only the edge bands
};

struct DescBatch {
  FrameDev f[kDescPerLaunch];
  int32_t first;
  int32_t count;
};

// Workspace header at offset 0 of every workspace.
struct QueueTotals {
  int64_t t[kQueues];
};

struct WsHeader {
  uint32_t error;        // bit 0: an index >= W*H was seen
  uint32_t pad0[15];
  struct {
    unsigned long long head;  // next item of this queue (own 64-byte line)
    uint64_t pad[7];
  } q[kQueues];
};
constexpr size_t kHeaderBytes = 1024;
static_assert(sizeof(WsHeader) <= kHeaderBytes, "header");

// Records `msg` as the calling thread's last error (sbs_last_error) and returns status.
int report_error(int status, const char* msg);

}  // namespace sbs
