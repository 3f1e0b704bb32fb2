/*
 * sbs.h - boundary-pixel SAD stereo disparity on AMD Instinct MI355X (gfx950).
 *
 * The operation (Mukherjee & Guddeti, arXiv 2001.07809, Sec. III "Disparity
 * Measurement of Boundary Pixels", with the winner-takes-all rule of Sec. II
 * and the O(N_b w^2 d) cost of the sequential complexity analysis):
 * for a rectified stereo pair the match of a left pixel lies on the same row
 * of the right image. Only the listed ("boundary") pixels are evaluated. For
 * list entry k, with p = idx[k], x = p mod W, y = p div W, r = (block-1)/2:
 *
 *   cost(d) = sum_{j=-r..r} sum_{i=-r..r} sum_{c<C}
 *             | L[cy(y+j)][cx(x+i)][c] - R[cy(y+j)][cx(x-d+i)][c] |
 *
 * for every d in 0..dmax, where cx and cy clamp to the image (replicate
 * padding, each coordinate on its own). out_disp[k] is the smallest d with the
 * least cost and out_cost[k] is that cost. Results are exact integers. They
 * depend only on (images, x, y, block, dmax), never on the rest of the list,
 * its order or batching.
 *
 * Conventions for every entry point:
 *  - Images are 8-bit, interleaved HWC (C = 1 gray or C = 3 RGB), rows
 *    pitch_bytes apart, pitch_bytes >= W*C. Image, list and output pointers
 *    are DEVICE memory owned by the caller. The library never frees them and
 *    keeps no pointer to them after the enqueued work completes.
 *  - Calls are asynchronous and ordered on `stream` (a hipStream_t; NULL is
 *    the null stream). A call returns once the work is enqueued. The caller
 *    keeps buffers alive until the stream reaches that point.
 *  - Arguments are checked on the host before any device work. The status is
 *    returned, never thrown; sbs_last_error() gives the message for the last
 *    non-OK status on the calling thread.
 *  - Indices must be < W*H. The kernels never read out of bounds. An index
 *    >= W*H yields out_disp 255 and out_cost 0xFFFFFFFF and sets a device
 *    error word that sbs_check_indices() reports as SBS_ERR_INDEX_RANGE.
 *  - Duplicated indices are allowed; n = 0 is a successful no-op.
 */
#ifndef SBS_H
#define SBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBS_ABI_VERSION 1

typedef enum {
  SBS_OK = 0,
  SBS_ERR_INVALID_ARG = 1, /* NULL pointer with n > 0, W or H < 1, C not 1 or 3,
                              pitch < W*C, block even or < 1, dmax < 0 or > 255,
                              n < 0, workspace too small for an explicit workspace */
  SBS_ERR_UNSUPPORTED = 2, /* block > SBS_MAX_BLOCK, or no gfx950 device */
  SBS_ERR_WORKSPACE = 3,   /* the library could not allocate its own workspace */
  SBS_ERR_HIP = 4,         /* a HIP runtime call failed; see sbs_last_error() */
  SBS_ERR_INDEX_RANGE = 5  /* an index >= W*H was seen (sbs_check_indices) */
} sbs_status;

/* Largest supported block (window side). The cost of a window must fit 24
 * bits: block^2 * C * 255 < 2^24. */
#define SBS_MAX_BLOCK 127

/*
 * Single frame. Computes out_disp[k] (and out_cost[k] unless out_cost is
 * NULL) for the n listed pixels.
 *   left, right    device, HWC u8, W x H x C, rows pitch_bytes apart
 *   boundary_idx   device, n entries, raster index y*W + x (any order)
 *   block          odd window side, 1..SBS_MAX_BLOCK
 *   dmax           largest disparity searched, 0..255 (dmax+1 candidates)
 *   out_disp       device, n bytes
 *   out_cost       device, n u32, or NULL
 *   workspace      device scratch of at least sbs_workspace_bytes() for this
 *                  one frame, or NULL with workspace_bytes 0 for a workspace
 *                  the library allocates, keeps and grows itself (that path
 *                  may allocate and is not safe under stream capture)
 *   stream         hipStream_t or NULL
 */
int sbs_sad_disparity(const uint8_t* left, const uint8_t* right, int32_t W, int32_t H, int32_t C,
                      int64_t pitch_bytes, const uint32_t* boundary_idx, int64_t n, int32_t block,
                      int32_t dmax, uint8_t* out_disp, uint32_t* out_cost, void* workspace,
                      size_t workspace_bytes, void* stream);

/*
 * For callers that cannot allocate (code under stream capture, serving loops
 * and harnesses that forbid allocation): sbs_sad_disparity for one frame,
 * computed in a fixed scratch array of SBS_SCRATCH_BYTES that the library
 * holds in device memory (one copy per GPU, from the library's first use on
 * that GPU until the process ends). The call allocates nothing and takes no
 * workspace; arguments, results and errors are those of sbs_sad_disparity,
 * plus SBS_ERR_WORKSPACE when the frame needs more than the scratch holds
 * (sbs_workspace_bytes for the frame > SBS_SCRATCH_BYTES; a 4096x2304 RGB
 * frame at block 31, dmax 127 and up to 100% listed pixels fits).
 * The first call on a device looks up that device's scratch address and
 * clears its header on `stream`; make that first call outside stream capture.
 * Every call on one GPU uses the same scratch: calls whose work overlaps on
 * one GPU (different streams, or host threads without ordering) race and
 * give wrong results; order them on one stream. Out-of-range indices are
 * answered with 255 / 0xFFFFFFFF as in sbs_sad_disparity; sbs_check_indices
 * does not read the scratch's error word.
 */
#define SBS_SCRATCH_BYTES (160u << 20)
int sbs_sad_disparity_noalloc(const uint8_t* left, const uint8_t* right, int32_t W, int32_t H, int32_t C,
                              int64_t pitch_bytes, const uint32_t* boundary_idx, int64_t n, int32_t block,
                              int32_t dmax, uint8_t* out_disp, uint32_t* out_cost, void* stream);

/* One frame of a batch. Field meanings as for sbs_sad_disparity. Host memory. */
typedef struct {
  const uint8_t* left;
  const uint8_t* right;
  int32_t W, H, C;
  int64_t pitch_bytes;
  const uint32_t* boundary_idx;
  int64_t n;
  int32_t block, dmax;
  uint8_t* out_disp;
  uint32_t* out_cost;
} sbs_frame;

/* Device workspace bytes needed by sbs_sad_disparity_batched for these
 * frames (and by sbs_sad_disparity for a single frame). 0 on invalid frames. */
size_t sbs_workspace_bytes(const sbs_frame* frames, int32_t nframes);

/*
 * Many frames in one pass: the per-frame work of every frame goes into one
 * work queue that a single persistent kernel drains (uneven boundary counts
 * and frame sizes balance across the GPU). Each frame's outputs equal what
 * sbs_sad_disparity gives for it alone.
 *   frames     host array of nframes descriptors (read during the call only;
 *              the descriptors travel to the device inside kernel arguments)
 *   workspace  device, >= sbs_workspace_bytes(frames, nframes), or NULL / 0
 *              for a library-managed workspace (not capture safe)
 * With an explicit workspace the call performs no allocation, no host
 * synchronisation and no copy from host memory, so it can be captured into a
 * hipGraph and replayed (replays recompute from the frames' current contents).
 */
int sbs_sad_disparity_batched(const sbs_frame* frames, int32_t nframes, void* workspace,
                              size_t workspace_bytes, void* stream);

/*
 * Debug check: synchronises `stream`, reads the device error word of
 * `workspace` (or of the library-managed workspace when NULL), clears it, and
 * returns SBS_ERR_INDEX_RANGE if any call since the last check saw an index
 * >= W*H, else SBS_OK. frames/nframes are accepted for symmetry and unused.
 */
int sbs_check_indices(const sbs_frame* frames, int32_t nframes, void* workspace, void* stream);

/*
 * Autotuner: times each tile plan (columns per lane, disparities per chunk,
 * rows per tile, persistent grid size) on these frames, keeps the fastest, and
 * stores it under the key (arch, W, H, C, block, dmax, density bucket,
 * frames per call rounded up to a power of two; taken from the first frame
 * with a non-empty list) in a JSON cache at cache_path (created or updated;
 * NULL: in memory only). Later calls with a matching key use the stored plan.
 * One frame is timed as sbs_sad_disparity runs it (one grid launch of the
 * tile kernel; the persistent grid size is then not searched), several
 * frames as sbs_sad_disparity_batched runs them.
 * Synchronous; runs in a library-managed workspace (allocated on first use,
 * kept until the process ends). Outputs of the frames are written as a side
 * effect.
 */
int sbs_tune(const sbs_frame* frames, int32_t nframes, const char* cache_path);

/* Loads a JSON tuning cache written by sbs_tune. Returns SBS_OK or SBS_ERR_INVALID_ARG. */
int sbs_load_tuning(const char* cache_path);

/* Message for the last non-OK status on the calling thread ("" if none). */
const char* sbs_last_error(void);

/* SBS_ABI_VERSION of the loaded library. */
int sbs_abi_version(void);

/*
 * Reference path: the same operation by direct brute force (one wavefront
 * per pixel, lanes over disparities, images read in place with clamped
 * coordinates), sharing no kernel with the tiled path. For cross-checks and
 * for parity tests; no workspace. Arguments as for sbs_sad_disparity.
 */
int sbs_sad_disparity_ref(const uint8_t* left, const uint8_t* right, int32_t W, int32_t H, int32_t C,
                          int64_t pitch_bytes, const uint32_t* boundary_idx, int64_t n, int32_t block,
                          int32_t dmax, uint8_t* out_disp, uint32_t* out_cost, void* stream);

/*
 * Per-frame launch path for the batching comparison: runs the frames one at a
 * time, each as its own sequence of launches on `stream` (no shared queue).
 * Same outputs as sbs_sad_disparity_batched. Workspace as for the batched call.
 */
int sbs_sad_disparity_per_frame(const sbs_frame* frames, int32_t nframes, void* workspace,
                                size_t workspace_bytes, void* stream);

/*
 * Plan control (used by the tuner and the benchmark). A plan is
 * (cols_per_lane, chunk, tile_rows, waves_per_cu); 0 in a field means
 * "automatic". sbs_set_plan forces a plan for subsequent calls (all fields 0
 * restores automatic choice); sbs_get_plan reports the plan the library would
 * use for a single-frame call on `frame`, sbs_get_plan_batched the plan of a
 * batched call on `frames`. Valid cols_per_lane: 4, 8 (8 only with chunk 8); chunk:
 * 8, 16; tile_rows: 8..256; waves_per_cu: 1..16. A frame runs with 8 columns
 * per lane only where its window sums allow packed 16-bit accumulators
 * (2 * block * 255 * C <= 65535) and min(n, (tile_rows - 1) * W) < 2^23;
 * other frames of the same call run with 4. A frame whose
 * min(n, (tile_rows - 1) * W) reaches 2^24 (2^23 at 8 columns per lane) runs
 * with tile_rows halved until it does not.
 */
typedef struct {
  int32_t cols_per_lane;
  int32_t chunk;
  int32_t tile_rows;
  int32_t waves_per_cu;
} sbs_plan;

int sbs_set_plan(const sbs_plan* plan);
int sbs_get_plan(const sbs_frame* frame, sbs_plan* plan);
int sbs_get_plan_batched(const sbs_frame* frames, int32_t nframes, sbs_plan* plan);

/*
 * Kernel timing (for the benchmark). While enabled, every call records a pair
 * of HIP events on its stream around each launch of the tile kernel (the
 * dominant kernel). sbs_kernel_times waits for the recorded pairs, writes up
 * to `cap` durations in milliseconds to `ms` (in launch order), releases them
 * and returns how many pairs there were. Not for use under stream capture.
 */
int sbs_kernel_timing(int32_t enable);
int32_t sbs_kernel_times(float* ms, int32_t cap);

/*
 * Issue-rate probe (diagnostic; not part of the disparity path): runs
 * `blocks` one-wavefront workgroups, each lane issuing trips * 128 v_sad_u8
 * (16 independent chains, 8 steps per trip) back to back, and reports the
 * v_sad_u8 lane operations per second and the kernel's duration (HIP events,
 * after one warm-up launch, on the null stream; synchronous). This is the
 * rate the tile kernel's integer-ALU roofline assumes: 256 CUs x 64 lanes
 * per clock. Allocates a small output buffer. SBS_ERR_INVALID_ARG for
 * blocks or trips < 1 or NULL outputs.
 */
int sbs_probe_sad_rate(int32_t blocks, int32_t trips, double* lane_ops_per_s, double* ms);

/*
 * Disparity map reconstruction (Sec. III "Disparity Map Reconstruction from
 * Boundaries"): the listed pixels' disparities are spread to a dense u8 map.
 * Stage 1 (Algorithm 1, fill along scan lines): in each row, every pixel
 * strictly between two consecutive listed pixels with equal disparity takes
 * that disparity. Stage 2 (Algorithm 2, peek): every pixel still undetermined
 * looks at the nearest determined pixel above and below in its column (in
 * stage 1's output); if their difference exceeds `threshold` it takes the
 * smaller, else their mean rounded half up; with only one of them it takes
 * that one; with none, 0. A repeated index keeps the disparity of its last
 * list entry; indices >= W*H are ignored.
 *   idx, disp   device, n entries (e.g. a list and the out_disp it produced)
 *   out_map     device, W*H bytes, row-major
 *   workspace   device, >= sbs_reconstruct_workspace_bytes(W, H)
 */
size_t sbs_reconstruct_workspace_bytes(int32_t W, int32_t H);
int sbs_reconstruct(const uint32_t* idx, const uint8_t* disp, int64_t n, int32_t W, int32_t H, int32_t threshold,
                    uint8_t* out_map, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Depth-based selective blurring (Sec. III, Eq. 1-2): a pixel whose depth
 * (disparity) lies outside every range of interest [lo_i, hi_i] is replaced,
 * per channel, by the convolution of the image with h = h_g / sum(h_g),
 * h_g(n1, n2) = exp(-(n1^2 + n2^2) / (2 sigma^2)), on a square support of side
 * 2 ceil(3 sigma) + 1 with replicate borders; other pixels keep their value.
 *   img         device, HWC u8, rows `pitch` bytes apart
 *   depth       device, W*H u8
 *   ranges      HOST array of nranges (lo, hi) pairs, nranges <= 16
 *   out         device, W*H*C float32, HWC, not rounded
 *   workspace   device, >= sbs_selective_blur_workspace_bytes(W, H, C), 4-byte
 *               aligned (radius <= 8 uses its first 12 bytes as a sink for
 *               stores outside the image; larger radii hold a float image)
 * Separable passes with fp32 sums. Radius ceil(3 sigma) <= 8: on the matrix
 * cores, taps and horizontal sums carried as fp16 high/low pairs, within
 * about 4e-4 of exact on outputs in [0, 255]; radius 9..64: fp32 taps on
 * the vector units. SBS_ERR_UNSUPPORTED if ceil(3 sigma) > 64.
 */
size_t sbs_selective_blur_workspace_bytes(int32_t W, int32_t H, int32_t C);
int sbs_selective_blur(const uint8_t* img, int32_t W, int32_t H, int32_t C, int64_t pitch, const uint8_t* depth,
                       const int32_t* ranges, int32_t nranges, float sigma, float* out, void* workspace,
                       size_t workspace_bytes, void* stream);

/*
 * Lightness (Sec. III, Colour Space Conversion): the L of CIE L*a*b* per
 * pixel, scaled to 8 bits. C == 3: sRGB decode of each channel, Y = 0.2126 R
 * + 0.7152 G + 0.0722 B on linear values, L* = 116 f(Y) - 16 with the CIE f
 * (cube root above (6/29)^3, linear below), L8 = round-half-away(L* 255/100),
 * in fp64 with every operation rounded on its own. C == 1: L8 = the gray value.
 *   img      device, HWC u8, rows `pitch` bytes apart (pitch >= W*C)
 *   out_l8   device, W*H bytes, row-major
 * Asynchronous on `stream`. SBS_ERR_INVALID_ARG for bad geometry or NULL.
 */
int sbs_lightness(const uint8_t* img, int32_t W, int32_t H, int32_t C, int64_t pitch, uint8_t* out_l8, void* stream);

/*
 * Refined segment-boundary pixels of the left image, the list the disparity
 * search runs on (Sec. III: Colour Space Conversion, Segmentation, Segment
 * Boundary Detection, Refinement; the border rule of Disparity Measurement).
 *   lightness -> 256-bin histogram -> K-means on the bins (distance |a - b|,
 *   exact rational centres, start c_k = Lmin + floor((2k+1)(Lmax-Lmin+1)/2K),
 *   ties to the lower cluster, empty clusters keep their centre, stop when no
 *   bin changes or after 1000 passes, clusters renumbered by ascending centre)
 *   -> label image ->
 *     mode 0 (configured): 3x3 open then close on the labels (replicate
 *       border), 8-neighbour boundary map, keep 8-connected components of at
 *       least min_cc pixels;
 *     mode 1 (paper): 8-neighbour boundary map, 'fill' (a 0 whose eight
 *       neighbours are 1 becomes 1), 'remove' (a 1 whose four 4-neighbours are
 *       1 becomes 0), both with outside pixels = 0; then drop the smallest
 *       8-connected components, ties by smallest raster index, while the
 *       dropped total stays <= floor(0.04 * all boundary pixels)
 *   -> list = left and right border columns plus the kept pixels, ascending.
 *   frac >= 0 (a benchmark knob, not the paper's): instead exactly
 *   llround(frac * W * H) pixels (at most W*H), ranked as (1) border columns by
 *   raster index, (2) kept pixels by component size descending, then raster
 *   index, (3) the other pixels by chessboard distance to (1)+(2) ascending,
 *   then h(i) = SplitMix64's output function of (i xor seed), then raster
 *   index; still ascending raster indices. frac < 0: no fraction control.
 *   img          device, HWC u8, rows `pitch` bytes apart; C = 1 or 3
 *   K            clusters, 1..64
 *   out_idx      device, capacity W*H u32: raster indices y*W + x, ascending
 *   out_count    device, one int64: the list length (written by the GPU, so
 *                the call stays asynchronous)
 *   out_refined  device W*H bytes or NULL: the kept boundary map (1/0),
 *                without the border columns
 *   out_labels   device W*H bytes or NULL: the label image the boundary map
 *                is taken from (after open/close in mode 0)
 *   workspace    device, >= sbs_boundaries_workspace_bytes(W, H) bytes,
 *                256-byte aligned (as hipMalloc returns); the library keeps
 *                nothing in it between calls
 * W*H <= 2^31 - 1 and H <= 262140 (else SBS_ERR_UNSUPPORTED). Asynchronous
 * on `stream`; SBS_ERR_INVALID_ARG for bad arguments (nothing is launched then).
 */
size_t sbs_boundaries_workspace_bytes(int32_t W, int32_t H);
int sbs_boundaries(const uint8_t* img, int32_t W, int32_t H, int32_t C, int64_t pitch, int32_t K, int32_t mode,
                   int32_t min_cc, double frac, uint64_t seed, uint32_t* out_idx, int64_t* out_count,
                   uint8_t* out_refined, uint8_t* out_labels, void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SBS_H */
