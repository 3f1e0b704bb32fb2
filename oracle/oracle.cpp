// Oracle: a plain, slow, obviously correct CPU implementation of what the
// boundary-pixel SAD disparity path computes, written from the paper
// (Mukherjee & Guddeti, "Depth-based Selective Blurring in Stereo Images Using
// Accelerated Framework", arXiv 2001.07809).
//
// THIS IS TEST INFRASTRUCTURE. Only the tests, the smoke check and the
// benchmark's CPU-baseline leg may load it. The HIP product path never calls
// it, includes it or links it, and it shares no code with that path.
//
// Contents (each function cites the passage it follows):
//   lightness            - Sec. III "Colour Space Conversion" (CIE L*)
//   histogram, k-means   - Sec. III "Segmentation"; Sec. III sequential
//                          complexity analysis (distance |a-b| on [0,255])
//   label open/close     - configured 3x3 morphology (see readings below)
//   boundary map         - Sec. III "Segment Boundary Detection" (Moore nbhd)
//   fill / remove        - Sec. III "Refinement" (the 3x3 fill pattern; the
//                          4-neighbour remove rule)
//   connected components - Sec. III "Refinement" and the CC complexity
//                          analysis (flood fill, sort by size)
//   border pixels        - Sec. III "Disparity Measurement" (left/right map
//                          borders count as boundary)
//   fraction control     - not in the paper; a benchmark knob
//   SAD-WTA              - Sec. III "Disparity Measurement" (same-row search,
//                          SAD cost), Sec. II (winner takes all), complexity
//                          O(N_b w^2 d)
//   dense SAT SAD        - a second, independent algorithm for the same SAD
//                          (summed-area table of the absolute-difference image)
//   reconstruction       - Sec. III Algorithm 1 (fill along scan lines) and
//                          Algorithm 2 (peek along columns)
//   selective blur       - Sec. III "Depth-based Selective Blurring", Eq. 1-2
//
// Readings of silent or ambiguous points are listed beside each function.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int oracle_version(void) { return 1; }

// ---------------------------------------------------------------------------
// Lightness (Sec. III, Colour Space Conversion). The paper keeps the 'L' of
// CIE Lab; its transform reference is lost. Reading: sRGB decode, D65
// luminance Y = 0.2126 R + 0.7152 G + 0.0722 B on linear values,
// L* = 116 f(Y) - 16 with the CIE f(), then L8 = round-half-away(L* 255/100).
// C == 1: the gray value is the lightness.
void oracle_lightness(const uint8_t* img, int32_t W, int32_t H, int32_t C,
                      int64_t pitch, uint8_t* L8) {
  double lin[256];
  for (int v = 0; v < 256; ++v) {
    double c = v / 255.0;
    lin[v] = c <= 0.04045 ? c / 12.92 : std::pow((c + 0.055) / 1.055, 2.4);
  }
  const double e = 6.0 / 29.0;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const uint8_t* p = img + (int64_t)y * pitch + (int64_t)x * C;
      if (C == 1) { L8[(int64_t)y * W + x] = p[0]; continue; }
      double Y = 0.2126 * lin[p[0]] + 0.7152 * lin[p[1]] + 0.0722 * lin[p[2]];
      double f = Y > e * e * e ? std::cbrt(Y) : Y / (3 * e * e) + 4.0 / 29.0;
      double Ls = 116.0 * f - 16.0;
      double s = Ls * 255.0 / 100.0;
      long q = (long)(s >= 0 ? std::floor(s + 0.5) : -std::floor(-s + 0.5));
      L8[(int64_t)y * W + x] = (uint8_t)clampi((int)q, 0, 255);
    }
}

// Histogram of lightness (Sec. III Segmentation: 256 bins).
void oracle_histogram(const uint8_t* L8, int64_t N, int64_t* hist) {
  for (int v = 0; v < 256; ++v) hist[v] = 0;
  for (int64_t i = 0; i < N; ++i) hist[L8[i]]++;
}

// K-means on histogram bins (Sec. III Segmentation; distance |a - b| between
// integers in [0, 255] from the sequential complexity analysis). Each
// occupied bin is a point weighted by its count; a pixel takes its bin's
// cluster. Readings: initial centres c_k = Lmin + floor((2k+1)(Lmax-Lmin+1)/(2K));
// centres are kept as exact rationals S_k/N_k; ties go to the lower k; an
// empty cluster keeps its centre; stop when no bin changes (at most 1000
// passes); finally clusters are renumbered by ascending centre.
// Outputs: bin_label[256] (-1 for empty bins) and centres as (S, N) pairs.
// Returns the number of assignment passes made.
int oracle_kmeans_bins(const int64_t* hist, int32_t K, int32_t* bin_label,
                       int64_t* cS, int64_t* cN) {
  int lo = -1, hi = -1;
  for (int b = 0; b < 256; ++b)
    if (hist[b] > 0) { if (lo < 0) lo = b; hi = b; }
  for (int b = 0; b < 256; ++b) bin_label[b] = -1;
  if (lo < 0 || K < 1) return 0;
  std::vector<int64_t> S(K), Nn(K);
  for (int k = 0; k < K; ++k) {
    S[k] = lo + ((int64_t)(2 * k + 1) * (hi - lo + 1)) / (2 * K);
    Nn[k] = 1;
  }
  std::vector<int> assign(256, -1);
  int pass = 0;
  for (; pass < 1000; ++pass) {
    bool changed = false;
    for (int b = lo; b <= hi; ++b) {
      if (hist[b] == 0) continue;
      int best = 0;
      for (int k = 1; k < K; ++k) {
        // |b - S_k/N_k| < |b - S_best/N_best|  <=>  |b N_k - S_k| N_best < |b N_best - S_best| N_k
        int64_t dk = std::llabs((int64_t)b * Nn[k] - S[k]);
        int64_t db = std::llabs((int64_t)b * Nn[best] - S[best]);
        if ((__int128)dk * Nn[best] < (__int128)db * Nn[k]) best = k;
      }
      if (assign[b] != best) { assign[b] = best; changed = true; }
    }
    if (!changed && pass > 0) break;
    std::vector<int64_t> s2(K, 0), n2(K, 0);
    for (int b = lo; b <= hi; ++b)
      if (hist[b] > 0) { s2[assign[b]] += (int64_t)b * hist[b]; n2[assign[b]] += hist[b]; }
    for (int k = 0; k < K; ++k)
      if (n2[k] > 0) { S[k] = s2[k]; Nn[k] = n2[k]; }
    if (!changed) break;
  }
  std::vector<int> order(K);
  for (int k = 0; k < K; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (__int128)S[a] * Nn[b] < (__int128)S[b] * Nn[a];
  });
  std::vector<int> rank(K);
  for (int i = 0; i < K; ++i) rank[order[i]] = i;
  for (int b = 0; b < 256; ++b) bin_label[b] = assign[b] < 0 ? -1 : rank[assign[b]];
  for (int i = 0; i < K; ++i) { cS[i] = S[order[i]]; cN[i] = Nn[order[i]]; }
  return pass + 1;
}

// Pixel labels from bin labels (Sec. III: one-to-one pixel-to-bin mapping).
void oracle_label_pixels(const uint8_t* L8, int64_t N, const int32_t* bin_label, uint8_t* lab) {
  for (int64_t i = 0; i < N; ++i) lab[i] = (uint8_t)std::max(0, bin_label[L8[i]]);
}

// 3x3 grayscale erosion (mode 0: min) or dilation (mode 1: max), replicate border.
static void morph3(const uint8_t* in, int W, int H, int mode, uint8_t* out) {
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int v = in[(int64_t)y * W + x];
      for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i) {
          int u = in[(int64_t)clampi(y + j, 0, H - 1) * W + clampi(x + i, 0, W - 1)];
          v = mode == 0 ? std::min(v, u) : std::max(v, u);
        }
      out[(int64_t)y * W + x] = (uint8_t)v;
    }
}

// Configured refinement: 3x3 open then close on the label image (labels are
// ordered by lightness). Reading: applied to labels, not to the boundary
// map, because a 3x3 opening would erase the two-pixel-wide 8-neighbour
// boundaries.
void oracle_label_open_close(const uint8_t* lab, int32_t W, int32_t H, uint8_t* out) {
  std::vector<uint8_t> a((size_t)W * H), b((size_t)W * H);
  morph3(lab, W, H, 0, a.data());      // erode
  morph3(a.data(), W, H, 1, b.data()); // dilate  -> open
  morph3(b.data(), W, H, 1, a.data()); // dilate
  morph3(a.data(), W, H, 0, out);      // erode   -> close
}

void oracle_erode3(const uint8_t* in, int32_t W, int32_t H, uint8_t* out) { morph3(in, W, H, 0, out); }
void oracle_dilate3(const uint8_t* in, int32_t W, int32_t H, uint8_t* out) { morph3(in, W, H, 1, out); }

// Boundary map (Sec. III Segment Boundary Detection): 1 iff some in-image
// Moore (8-) neighbour has a different label.
void oracle_boundary(const uint8_t* lab, int32_t W, int32_t H, uint8_t* B) {
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      uint8_t v = lab[(int64_t)y * W + x], m = 0;
      for (int j = -1; j <= 1 && !m; ++j)
        for (int i = -1; i <= 1; ++i) {
          int yy = y + j, xx = x + i;
          if ((i || j) && yy >= 0 && yy < H && xx >= 0 && xx < W && lab[(int64_t)yy * W + xx] != v) { m = 1; break; }
        }
      B[(int64_t)y * W + x] = m;
    }
}

// 'Fill' (Sec. III Refinement): a 0 whose eight neighbours are all 1 becomes 1
// (the printed 3x3 pattern). Reading: computed from the whole previous map;
// out-of-image neighbours count as 0.
void oracle_fill(const uint8_t* B, int32_t W, int32_t H, uint8_t* out) {
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      uint8_t v = B[(int64_t)y * W + x];
      if (!v) {
        bool all = true;
        for (int j = -1; j <= 1 && all; ++j)
          for (int i = -1; i <= 1; ++i) {
            if (!i && !j) continue;
            int yy = y + j, xx = x + i;
            if (yy < 0 || yy >= H || xx < 0 || xx >= W || !B[(int64_t)yy * W + xx]) { all = false; break; }
          }
        if (all) v = 1;
      }
      out[(int64_t)y * W + x] = v;
    }
}

// 'Remove' (Sec. III Refinement): a 1 whose four 4-connected neighbours are
// all 1 becomes 0. Same reading as fill.
void oracle_remove(const uint8_t* B, int32_t W, int32_t H, uint8_t* out) {
  auto at = [&](int yy, int xx) -> int {
    return (yy < 0 || yy >= H || xx < 0 || xx >= W) ? 0 : B[(int64_t)yy * W + xx];
  };
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      uint8_t v = B[(int64_t)y * W + x];
      if (v && at(y - 1, x) && at(y + 1, x) && at(y, x - 1) && at(y, x + 1)) v = 0;
      out[(int64_t)y * W + x] = v;
    }
}

// 8-connected components of a binary map (Sec. III: scan for an unlabelled
// pixel, flood fill its component; repeat). The flood fill uses an explicit
// stack instead of recursion. Components are numbered 0.. in the order the
// raster scan finds them (so by their smallest raster index).
// comp[i] = component of pixel i or -1. Returns the count; sizes[] (capacity
// W*H) receives each component's pixel count.
int64_t oracle_components(const uint8_t* B, int32_t W, int32_t H, int32_t* comp, int64_t* sizes) {
  const int64_t N = (int64_t)W * H;
  for (int64_t i = 0; i < N; ++i) comp[i] = -1;
  int64_t nc = 0;
  std::vector<int64_t> stack;
  for (int64_t s = 0; s < N; ++s) {
    if (!B[s] || comp[s] >= 0) continue;
    int64_t size = 0;
    comp[s] = (int32_t)nc;
    stack.push_back(s);
    while (!stack.empty()) {
      int64_t q = stack.back();
      stack.pop_back();
      ++size;
      int y = (int)(q / W), x = (int)(q % W);
      for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i) {
          int yy = y + j, xx = x + i;
          if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
          int64_t t = (int64_t)yy * W + xx;
          if (B[t] && comp[t] < 0) { comp[t] = (int32_t)nc; stack.push_back(t); }
        }
    }
    sizes[nc++] = size;
  }
  return nc;
}

// Component filter. mode 0 (configured): keep components with at least
// min_size pixels. mode 1 (the paper's rule, Sec. III Refinement): order
// components by size (ties: by smallest raster index) and drop the smallest
// ones while the dropped total stays within drop_frac of all boundary pixels.
// Writes the kept map to out.
void oracle_cc_filter(const uint8_t* B, int32_t W, int32_t H, int32_t mode, int64_t min_size,
                      double drop_frac, uint8_t* out) {
  const int64_t N = (int64_t)W * H;
  std::vector<int32_t> comp((size_t)N);
  std::vector<int64_t> sizes((size_t)N + 1);
  int64_t nc = oracle_components(B, W, H, comp.data(), sizes.data());
  std::vector<uint8_t> keep((size_t)nc + 1, 1);
  if (mode == 0) {
    for (int64_t c = 0; c < nc; ++c) keep[(size_t)c] = sizes[(size_t)c] >= min_size;
  } else {
    int64_t total = 0;
    for (int64_t c = 0; c < nc; ++c) total += sizes[(size_t)c];
    std::vector<int64_t> ord((size_t)nc);
    for (int64_t c = 0; c < nc; ++c) ord[(size_t)c] = c;
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return sizes[(size_t)a] < sizes[(size_t)b]; });
    int64_t dropped = 0;
    for (int64_t c : ord) {
      if ((double)(dropped + sizes[(size_t)c]) > drop_frac * (double)total) break;
      dropped += sizes[(size_t)c];
      keep[(size_t)c] = 0;
    }
  }
  for (int64_t i = 0; i < N; ++i) out[i] = (uint8_t)(comp[(size_t)i] >= 0 && keep[(size_t)comp[(size_t)i]]);
}

// Border columns plus refined pixels, then optional fraction control (the
// last step of the front end; Sec. III: pixels that map to the left/right
// borders of the disparity map are boundary pixels too).
// refined: W*H map (1 = kept boundary pixel).
// frac < 0: the list is the border columns and the refined pixels.
// frac >= 0 (a benchmark knob, not the paper's): exactly round(frac*W*H)
// pixels ranked as (1) border columns, (2) refined pixels by component size
// descending then raster index, (3) other pixels by chessboard distance to
// the set of (1)+(2) ascending, then mix64(index ^ seed), then index.
// Output: ascending raster indices. Returns the count, -1 on error.
int64_t oracle_fraction_select(const uint8_t* refined, int32_t W, int32_t H, double frac, uint64_t seed,
                               uint32_t* out, int64_t cap) {
  if (W < 1 || H < 1) return -1;
  const int64_t N = (int64_t)W * H;
  const uint8_t* R = refined;
  std::vector<uint8_t> sel((size_t)N, 0);
  for (int y = 0; y < H; ++y) { sel[(size_t)y * W] = 1; sel[(size_t)y * W + W - 1] = 1; }
  if (frac < 0) {
    int64_t n = 0;
    for (int64_t i = 0; i < N; ++i)
      if (sel[(size_t)i] || R[(size_t)i]) { if (n >= cap) return -1; out[n++] = (uint32_t)i; }
    return n;
  }
  const int64_t want = std::min<int64_t>(N, std::llround(frac * (double)N));
  if (want > cap) return -1;
  // Rank keys: (class, primary, secondary) compared lexicographically.
  std::vector<int32_t> comp((size_t)N);
  std::vector<int64_t> sizes((size_t)N + 1);
  oracle_components(R, W, H, comp.data(), sizes.data());
  // Chessboard distance to the selected set: two raster passes, each taking
  // the 8-neighbours already visited (exact for this metric).
  const int32_t INF = 1 << 28;
  std::vector<int32_t> dist((size_t)N, INF);
  for (int64_t i = 0; i < N; ++i) if (sel[(size_t)i] || R[(size_t)i]) dist[(size_t)i] = 0;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int32_t& d = dist[(size_t)y * W + x];
      if (x > 0) d = std::min(d, dist[(size_t)y * W + x - 1] + 1);
      if (y > 0)
        for (int i = -1; i <= 1; ++i)
          if (x + i >= 0 && x + i < W) d = std::min(d, dist[(size_t)(y - 1) * W + x + i] + 1);
    }
  for (int y = H - 1; y >= 0; --y)
    for (int x = W - 1; x >= 0; --x) {
      int32_t& d = dist[(size_t)y * W + x];
      if (x + 1 < W) d = std::min(d, dist[(size_t)y * W + x + 1] + 1);
      if (y + 1 < H)
        for (int i = -1; i <= 1; ++i)
          if (x + i >= 0 && x + i < W) d = std::min(d, dist[(size_t)(y + 1) * W + x + i] + 1);
    }
  struct Key { int32_t cls; int64_t a; uint64_t b; int64_t idx; };
  std::vector<Key> keys((size_t)N);
  for (int64_t i = 0; i < N; ++i) {
    Key k;
    k.idx = i;
    if (sel[(size_t)i]) { k.cls = 0; k.a = 0; k.b = (uint64_t)i; }
    else if (R[(size_t)i]) { k.cls = 1; k.a = -sizes[(size_t)comp[(size_t)i]]; k.b = (uint64_t)i; }
    else { k.cls = 2; k.a = dist[(size_t)i]; k.b = mix64((uint64_t)i ^ seed); }
    keys[(size_t)i] = k;
  }
  auto less = [](const Key& p, const Key& q) {
    if (p.cls != q.cls) return p.cls < q.cls;
    if (p.a != q.a) return p.a < q.a;
    if (p.b != q.b) return p.b < q.b;
    return p.idx < q.idx;
  };
  if (want < N) std::nth_element(keys.begin(), keys.begin() + want, keys.end(), less);
  std::vector<uint8_t> take((size_t)N, 0);
  for (int64_t i = 0; i < want; ++i) take[(size_t)keys[(size_t)i].idx] = 1;
  int64_t n = 0;
  for (int64_t i = 0; i < N; ++i) if (take[(size_t)i]) out[n++] = (uint32_t)i;
  return n;
}

// Full front end (Sec. III): lightness -> histogram K-means -> labels ->
// refinement -> boundary -> component filter -> oracle_fraction_select.
//   mode 0 (configured): label open/close, 8-neighbour boundary, keep CC >= min_cc.
//   mode 1 (paper): 8-neighbour boundary, fill, remove, drop smallest CCs
//                   totalling <= 4% of boundary pixels.
// frac and seed as for oracle_fraction_select. refined_map (W*H or NULL)
// receives the kept boundary map. Returns the count, -1 on error.
int64_t oracle_boundaries(const uint8_t* img, int32_t W, int32_t H, int32_t C, int64_t pitch,
                          int32_t K, int32_t mode, int64_t min_cc, double frac, uint64_t seed,
                          uint32_t* out, int64_t cap, uint8_t* refined_map) {
  if (W < 1 || H < 1 || (C != 1 && C != 3) || K < 1) return -1;
  const int64_t N = (int64_t)W * H;
  std::vector<uint8_t> L((size_t)N), lab((size_t)N), lab2((size_t)N), B((size_t)N), B2((size_t)N), R((size_t)N);
  oracle_lightness(img, W, H, C, pitch, L.data());
  int64_t hist[256];
  oracle_histogram(L.data(), N, hist);
  int32_t bl[256];
  std::vector<int64_t> cS(K), cN(K);
  oracle_kmeans_bins(hist, K, bl, cS.data(), cN.data());
  oracle_label_pixels(L.data(), N, bl, lab.data());
  if (mode == 0) {
    oracle_label_open_close(lab.data(), W, H, lab2.data());
    oracle_boundary(lab2.data(), W, H, B.data());
    oracle_cc_filter(B.data(), W, H, 0, min_cc, 0.0, R.data());
  } else {
    oracle_boundary(lab.data(), W, H, B.data());
    oracle_fill(B.data(), W, H, B2.data());
    oracle_remove(B2.data(), W, H, B.data());
    oracle_cc_filter(B.data(), W, H, 1, 0, 0.04, R.data());
  }
  if (refined_map) std::memcpy(refined_map, R.data(), (size_t)N);
  return oracle_fraction_select(R.data(), W, H, frac, seed, out, cap);
}

// ---------------------------------------------------------------------------
// SAD-WTA at listed pixels (Sec. III Disparity Measurement; Sec. II WTA).
// For list entry k: p = idx[k], x = p mod W, y = p div W, r = (block-1)/2,
//   cost(d) = sum_{j=-r..r} sum_{i=-r..r} sum_{c<C}
//             | L[cy(y+j)][cx(x+i)][c] - R[cy(y+j)][cx(x-d+i)][c] |
// for d = 0..dmax, where cx, cy clamp to the image (replicate padding, each
// coordinate on its own). The match is searched to the left in the right
// image (x - d) on the same row. The first d with the smallest cost wins
// (strict '<' while d increases, so ties go to the smaller d).
// Outputs disp[k] = d*, cost[k] = cost(d*). An index >= W*H gives disp 255,
// cost 0xFFFFFFFF and makes the return value 5; otherwise 0.
// Images: HWC u8 with row pitch in bytes. OpenMP over the list.
int oracle_sad(const uint8_t* left, const uint8_t* right, int32_t W, int32_t H, int32_t C,
               int64_t pitch, const uint32_t* idx, int64_t n, int32_t block, int32_t dmax,
               uint8_t* disp, uint32_t* cost, int32_t threads) {
  if (W < 1 || H < 1 || (C != 1 && C != 3) || block < 1 || block % 2 == 0 || dmax < 0 || dmax > 255 || n < 0)
    return 1;
  const int r = (block - 1) / 2;
  const int64_t N = (int64_t)W * H;
  int bad = 0;
  if (threads < 1) threads = 1;
#pragma omp parallel for schedule(dynamic, 64) num_threads(threads) reduction(| : bad)
  for (int64_t k = 0; k < n; ++k) {
    const int64_t p = idx[k];
    if (p >= N) { disp[k] = 255; cost[k] = 0xFFFFFFFFu; bad = 1; continue; }
    const int x = (int)(p % W), y = (int)(p / W);
    uint32_t best = 0xFFFFFFFFu;
    int bd = 0;
    for (int d = 0; d <= dmax; ++d) {
      uint32_t s = 0;
      for (int j = -r; j <= r; ++j) {
        const int yy = clampi(y + j, 0, H - 1);
        const uint8_t* Lrow = left + (int64_t)yy * pitch;
        const uint8_t* Rrow = right + (int64_t)yy * pitch;
        for (int i = -r; i <= r; ++i) {
          const uint8_t* a = Lrow + (int64_t)clampi(x + i, 0, W - 1) * C;
          const uint8_t* b = Rrow + (int64_t)clampi(x - d + i, 0, W - 1) * C;
          for (int c = 0; c < C; ++c) s += (uint32_t)std::abs((int)a[c] - (int)b[c]);
        }
      }
      if (s < best) { best = s; bd = d; }
    }
    disp[k] = (uint8_t)bd;
    cost[k] = best;
  }
  return bad ? 5 : 0;
}

// The same SAD-WTA by a different algorithm: for each d, the absolute-
// difference image over the replicate-padded domain is summed into a
// summed-area table and each window is read as four table entries.
// Used only to cross-check oracle_sad. Same outputs and return codes.
int oracle_sad_sat(const uint8_t* left, const uint8_t* right, int32_t W, int32_t H, int32_t C,
                   int64_t pitch, const uint32_t* idx, int64_t n, int32_t block, int32_t dmax,
                   uint8_t* disp, uint32_t* cost) {
  if (W < 1 || H < 1 || (C != 1 && C != 3) || block < 1 || block % 2 == 0 || dmax < 0 || dmax > 255 || n < 0)
    return 1;
  const int r = (block - 1) / 2;
  const int64_t N = (int64_t)W * H;
  const int PW = W + 2 * r, PH = H + 2 * r;  // padded domain: columns -r..W-1+r, rows -r..H-1+r
  std::vector<uint32_t> best((size_t)n, 0xFFFFFFFFu);
  std::vector<uint8_t> bd((size_t)n, 0);
  std::vector<int64_t> S((size_t)(PW + 1) * (PH + 1));
  int bad = 0;
  for (int d = 0; d <= dmax; ++d) {
    for (int v = 0; v <= PH; ++v) S[(size_t)v * (PW + 1)] = 0;
    for (int u = 0; u <= PW; ++u) S[(size_t)u] = 0;
    for (int v = 0; v < PH; ++v) {
      const int yy = clampi(v - r, 0, H - 1);
      int64_t rowsum = 0;
      for (int u = 0; u < PW; ++u) {
        const int xa = clampi(u - r, 0, W - 1), xb = clampi(u - r - d, 0, W - 1);
        int64_t ad = 0;
        for (int c = 0; c < C; ++c)
          ad += std::abs((int)left[(int64_t)yy * pitch + (int64_t)xa * C + c] -
                         (int)right[(int64_t)yy * pitch + (int64_t)xb * C + c]);
        rowsum += ad;
        S[(size_t)(v + 1) * (PW + 1) + (u + 1)] = S[(size_t)v * (PW + 1) + (u + 1)] + rowsum;
      }
    }
    for (int64_t k = 0; k < n; ++k) {
      const int64_t p = idx[k];
      if (p >= N) continue;
      const int x = (int)(p % W), y = (int)(p / W);
      // window in padded coords: columns x..x+2r, rows y..y+2r
      const int64_t u0 = x, u1 = x + 2 * r + 1, v0 = y, v1 = y + 2 * r + 1;
      const int64_t s = S[(size_t)v1 * (PW + 1) + u1] - S[(size_t)v0 * (PW + 1) + u1] -
                        S[(size_t)v1 * (PW + 1) + u0] + S[(size_t)v0 * (PW + 1) + u0];
      if ((uint32_t)s < best[(size_t)k]) { best[(size_t)k] = (uint32_t)s; bd[(size_t)k] = (uint8_t)d; }
    }
  }
  for (int64_t k = 0; k < n; ++k) {
    if ((int64_t)idx[k] >= N) { disp[k] = 255; cost[k] = 0xFFFFFFFFu; bad = 1; }
    else { disp[k] = bd[(size_t)k]; cost[k] = best[(size_t)k]; }
  }
  return bad ? 5 : 0;
}

// ---------------------------------------------------------------------------
// Disparity map reconstruction (Sec. III).
// Input: the sparse map (disparity per listed pixel). Output dense u8 map.
// Stage 1, Algorithm 1 (fill along scan lines): in each row, left to right,
// when a boundary pixel has the same disparity as the previous boundary
// pixel of that row, every pixel strictly between them takes that value.
// Stage 2, Algorithm 2 (peek): every pixel still undetermined looks at the
// nearest determined pixel above and the nearest below in its column (as left
// by stage 1); if their range exceeds `threshold` it takes the smaller value,
// else their mean rounded half up. Readings: "two nearest" means the nearest
// above and the nearest below; with only one of them it takes that one; with
// none it takes 0; stage 2 reads only stage 1's output.
// Entries with an index >= W*H are ignored; a repeated index keeps its last value.
void oracle_reconstruct(const uint32_t* idx, const uint8_t* disp, int64_t n, int32_t W, int32_t H,
                        int32_t threshold, uint8_t* out) {
  const int64_t N = (int64_t)W * H;
  std::vector<int16_t> m((size_t)N, -1);
  std::vector<uint8_t> isb((size_t)N, 0);
  for (int64_t k = 0; k < n; ++k)
    if ((int64_t)idx[k] < N) { m[idx[k]] = disp[k]; isb[idx[k]] = 1; }
  std::vector<int16_t> f = m;  // after stage 1
  for (int y = 0; y < H; ++y) {
    int prev = -1;
    for (int x = 0; x < W; ++x) {
      const int64_t q = (int64_t)y * W + x;
      if (!isb[(size_t)q]) continue;
      if (prev >= 0 && m[(size_t)q] == m[(size_t)y * W + prev])
        for (int t = prev + 1; t < x; ++t) f[(size_t)y * W + t] = m[(size_t)q];
      prev = x;
    }
  }
  for (int x = 0; x < W; ++x)
    for (int y = 0; y < H; ++y) {
      const int64_t q = (int64_t)y * W + x;
      if (f[(size_t)q] >= 0) { out[q] = (uint8_t)f[(size_t)q]; continue; }
      int up = -1, dn = -1;
      for (int t = y - 1; t >= 0; --t) if (f[(size_t)t * W + x] >= 0) { up = f[(size_t)t * W + x]; break; }
      for (int t = y + 1; t < H; ++t) if (f[(size_t)t * W + x] >= 0) { dn = f[(size_t)t * W + x]; break; }
      int v;
      if (up < 0 && dn < 0) v = 0;
      else if (up < 0) v = dn;
      else if (dn < 0) v = up;
      else if (std::abs(up - dn) > threshold) v = std::min(up, dn);
      else v = (up + dn + 1) / 2;
      out[q] = (uint8_t)v;
    }
}

// ---------------------------------------------------------------------------
// Depth-based selective blurring (Sec. III, Eq. 1-2). A pixel is blurred iff
// its disparity lies outside every range of interest [lo_i, hi_i]. The
// kernel is h = h_g / sum(h_g) with h_g(n1, n2) = exp(-(n1^2 + n2^2) / (2 sigma^2))
// on a (2 ceil(3 sigma) + 1)^2 support (reading: the paper leaves the size
// open), replicate border (reading). Blurred pixels get the weighted sum per
// channel, in double; other pixels keep their value. Output: float per
// channel, HWC, not rounded.
void oracle_blur(const uint8_t* img, int32_t W, int32_t H, int32_t C, int64_t pitch,
                 const uint8_t* depth, const int32_t* ranges, int32_t nranges, double sigma,
                 float* out) {
  const int rad = (int)std::ceil(3.0 * sigma);
  const int K = 2 * rad + 1;
  std::vector<double> h((size_t)K * K);
  double hs = 0;
  for (int j = -rad; j <= rad; ++j)
    for (int i = -rad; i <= rad; ++i) {
      double g = std::exp(-(double)(i * i + j * j) / (2.0 * sigma * sigma));
      h[(size_t)(j + rad) * K + (i + rad)] = g;
      hs += g;
    }
  for (auto& v : h) v /= hs;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int dv = depth[(int64_t)y * W + x];
      bool keep = false;
      for (int t = 0; t < nranges; ++t)
        if (dv >= ranges[2 * t] && dv <= ranges[2 * t + 1]) { keep = true; break; }
      for (int c = 0; c < C; ++c) {
        double v;
        if (keep) v = img[(int64_t)y * pitch + (int64_t)x * C + c];
        else {
          v = 0;
          for (int j = -rad; j <= rad; ++j)
            for (int i = -rad; i <= rad; ++i)
              v += h[(size_t)(j + rad) * K + (i + rad)] *
                   img[(int64_t)clampi(y + j, 0, H - 1) * pitch + (int64_t)clampi(x + i, 0, W - 1) * C + c];
        }
        out[((int64_t)y * W + x) * C + c] = (float)v;
      }
    }
}

}  // extern "C"
