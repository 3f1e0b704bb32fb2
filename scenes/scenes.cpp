// Seeded synthetic stereo scenes.
//
// This module is the input generator shared by the tests, the benchmark and
// the oracle's checks. It makes rectified stereo pairs of textured, fronto-
// parallel regions with known integer disparity, a ground-truth map, an
// occlusion mask, the region-id map, and a list of pixels that lie near the
// scene's region outlines (the stand-in for a refined boundary set).
// It holds none of the disparity method's arithmetic: no lightness, no
// clustering, no boundary refinement, no matching cost.
//
// Random numbers: splitmix64 (Steele, Lea & Flood 2014) seeds xoshiro256**
// (Blackman & Vigna 2018) streams, one stream per (seed, purpose, id, row), so
// every value is independent of the number of threads used to make it.
// Integer ranges use rejection sampling; Gaussians use the Box-Muller method.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

inline uint64_t splitmix_next(uint64_t& s) {
  s += 0x9E3779B97F4A7C15ULL;
  return mix64(s);
}

inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

struct Rng {
  uint64_t s[4];
  Rng(uint64_t seed, uint64_t purpose, uint64_t id, uint64_t row) {
    uint64_t h = seed;
    h = mix64(h ^ (purpose * 0x9E3779B97F4A7C15ULL + 1));
    h = mix64(h ^ (id * 0xD1B54A32D192ED03ULL + 2));
    h = mix64(h ^ (row * 0x8CB92BA72F3D8DD7ULL + 3));
    for (int i = 0; i < 4; ++i) s[i] = splitmix_next(h);
  }
  uint64_t next() {
    const uint64_t result = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
  }
  // Uniform integer in [lo, hi] by rejection (no modulo bias).
  int64_t uniform(int64_t lo, int64_t hi) {
    if (hi <= lo) return lo;
    const uint64_t range = (uint64_t)(hi - lo) + 1;
    const uint64_t limit = UINT64_MAX - (UINT64_MAX % range);
    uint64_t x;
    do { x = next(); } while (x >= limit);
    return lo + (int64_t)(x % range);
  }
  double unit() { return (double)(next() >> 11) * 0x1.0p-53; }
};

// Box-Muller pairs, consumed in order (cos term, then sin term).
struct Gauss {
  Rng& r;
  bool have = false;
  double spare = 0.0;
  explicit Gauss(Rng& rr) : r(rr) {}
  double next() {
    if (have) { have = false; return spare; }
    double u1 = ((double)(r.next() >> 11) + 1.0) * 0x1.0p-53;  // (0, 1]
    double u2 = r.unit();
    double m = std::sqrt(-2.0 * std::log(u1));
    spare = m * std::sin(2.0 * M_PI * u2);
    have = true;
    return m * std::cos(2.0 * M_PI * u2);
  }
};

enum Purpose : uint64_t {
  P_LAYOUT = 1, P_BG_TEX = 2, P_REG_TEX = 3, P_RIGHT = 4,
  P_NOISE_L = 5, P_NOISE_R = 6, P_MOTION = 7, P_BG_MEAN = 8,
};

inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
inline uint8_t clamp_u8(long v) { return (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v)); }

}  // namespace

extern "C" {

typedef struct {
  int32_t W, H, C;          // image size; C is 1 (gray) or 3 (RGB)
  int32_t n_regions;        // number of foreground regions
  int32_t dmax_regions;     // region disparities are drawn from [0, dmax_regions]
  int32_t texture;          // 0: uniform noise smoothed by a 3x3 box; 1: Gaussian sigma 1
  int32_t mean_shift;       // 1: each region (and the background) gets a mean in [30, 225]
  int32_t ramp;             // 1: region 0 carries a horizontal disparity ramp of 0..8
  int32_t motion;           // per-frame position step is drawn from [-motion, motion]^2
  int32_t drift;            // per-frame disparity step is drawn from [-drift, drift]
  double noise_sigma;       // additive Gaussian noise on both images (0: none)
  uint64_t seed;
} sc_params;

}  // extern "C"

namespace {

struct Region {
  int shape;    // 0 rectangle, 1 ellipse
  int wr, hr;
  int cx, cy;
  int disp;     // base disparity (the ramp adds 0..8 on top)
  int mean;     // -1: none
};

// Uniform u8 noise, smoothed, optionally moved to a mean; HWC layout.
void make_texture(const sc_params& p, uint64_t purpose, uint64_t id, int w, int h,
                  int mean, std::vector<uint8_t>& out) {
  const int C = p.C;
  std::vector<uint8_t> noise((size_t)w * h * C);
#pragma omp parallel for schedule(static) if ((size_t)w * h > (1u << 18))
  for (int v = 0; v < h; ++v) {
    Rng r(p.seed, purpose, id, (uint64_t)v);
    uint8_t* row = &noise[(size_t)v * w * C];
    size_t n = (size_t)w * C, i = 0;
    while (i < n) {
      uint64_t x = r.next();
      for (int b = 0; b < 8 && i < n; ++b, ++i) row[i] = (uint8_t)(x >> (8 * b));
    }
  }
  out.assign((size_t)w * h * C, 0);
  if (p.texture == 0) {
    // 3x3 box, replicate border, integer (sum + 4) / 9, as row sums then column sums.
    std::vector<uint16_t> hs((size_t)w * h * C);
#pragma omp parallel for schedule(static) if ((size_t)w * h > (1u << 18))
    for (int v = 0; v < h; ++v) {
      const uint8_t* row = &noise[(size_t)v * w * C];
      uint16_t* o = &hs[(size_t)v * w * C];
      for (int u = 0; u < w; ++u) {
        const int ul = u > 0 ? u - 1 : 0, ur = u + 1 < w ? u + 1 : w - 1;
        for (int c = 0; c < C; ++c)
          o[(size_t)u * C + c] = (uint16_t)(row[(size_t)ul * C + c] + row[(size_t)u * C + c] + row[(size_t)ur * C + c]);
      }
    }
#pragma omp parallel for schedule(static) if ((size_t)w * h > (1u << 18))
    for (int v = 0; v < h; ++v) {
      const uint16_t* a = &hs[(size_t)clampi(v - 1, 0, h - 1) * w * C];
      const uint16_t* b = &hs[(size_t)v * w * C];
      const uint16_t* c2 = &hs[(size_t)clampi(v + 1, 0, h - 1) * w * C];
      uint8_t* o = &out[(size_t)v * w * C];
      for (size_t i = 0; i < (size_t)w * C; ++i) o[i] = (uint8_t)((a[i] + b[i] + c2[i] + 4) / 9);
    }
  } else {
    // Separable Gaussian, sigma 1, radius 3, fixed-point weights summing to 2^16.
    double g[7], gs = 0;
    for (int k = -3; k <= 3; ++k) { g[k + 3] = std::exp(-0.5 * k * k); gs += g[k + 3]; }
    int64_t wt[7], ws = 0;
    for (int k = 0; k < 7; ++k) { wt[k] = (int64_t)std::llround(g[k] / gs * 65536.0); ws += wt[k]; }
    wt[3] += 65536 - ws;
    std::vector<uint32_t> tmp((size_t)w * h * C);
#pragma omp parallel for schedule(static) if ((size_t)w * h > (1u << 18))
    for (int v = 0; v < h; ++v)
      for (int u = 0; u < w; ++u)
        for (int c = 0; c < C; ++c) {
          int64_t s = 0;
          for (int k = -3; k <= 3; ++k)
            s += wt[k + 3] * noise[((size_t)v * w + clampi(u + k, 0, w - 1)) * C + c];
          tmp[((size_t)v * w + u) * C + c] = (uint32_t)s;
        }
#pragma omp parallel for schedule(static) if ((size_t)w * h > (1u << 18))
    for (int v = 0; v < h; ++v)
      for (int u = 0; u < w; ++u)
        for (int c = 0; c < C; ++c) {
          uint64_t s = 0;
          for (int k = -3; k <= 3; ++k)
            s += (uint64_t)wt[k + 3] * tmp[((size_t)clampi(v + k, 0, h - 1) * w + u) * C + c];
          out[((size_t)v * w + u) * C + c] = (uint8_t)std::min<uint64_t>(255, (s + (1ULL << 31)) >> 32);
        }
  }
  if (mean >= 0) {
    for (auto& t : out) {
      int s = (int)t - 128;
      int half = s >= 0 ? s / 2 : -((-s + 1) / 2);  // floor(s / 2)
      t = clamp_u8(mean + half);
    }
  }
}

std::vector<Region> layout(const sc_params& p, int frame, int* bg_mean) {
  Rng r(p.seed, P_LAYOUT, 0, 0);
  const int W = p.W, H = p.H, D = p.dmax_regions;
  std::vector<Region> reg((size_t)std::max(0, p.n_regions));
  for (int k = 0; k < p.n_regions; ++k) {
    Region& g = reg[k];
    g.shape = (int)r.uniform(0, 1);
    g.wr = (int)r.uniform(std::max(2, W / 16), std::max(2, W / 4));
    g.hr = (int)r.uniform(std::max(2, H / 16), std::max(2, H / 4));
    g.cx = (int)r.uniform(0, W - 1);
    g.cy = (int)r.uniform(0, H - 1);
    if (p.ramp && k == 0) g.disp = (int)r.uniform(0, std::max(0, D - 8));
    else g.disp = (int)r.uniform(0, D);
    g.mean = p.mean_shift ? (int)r.uniform(30, 225) : -1;
  }
  {
    Rng rb(p.seed, P_BG_MEAN, 0, 0);
    *bg_mean = p.mean_shift ? (int)rb.uniform(30, 225) : -1;
  }
  // Video: positions and disparities follow a seeded random walk.
  for (int t = 1; t <= frame; ++t) {
    Rng m(p.seed, P_MOTION, (uint64_t)t, 0);
    for (int k = 0; k < p.n_regions; ++k) {
      Region& g = reg[k];
      int dx = (int)m.uniform(-p.motion, p.motion);
      int dy = (int)m.uniform(-p.motion, p.motion);
      int dd = (int)m.uniform(-p.drift, p.drift);
      g.cx = clampi(g.cx + dx, 0, W - 1);
      g.cy = clampi(g.cy + dy, 0, H - 1);
      int dhi = (p.ramp && k == 0) ? std::max(0, D - 8) : D;
      g.disp = clampi(g.disp + dd, 0, dhi);
    }
  }
  return reg;
}

inline bool inside_ellipse(int u, int v, int wr, int hr) {
  // (2u + 1 - wr)^2 / wr^2 + (2v + 1 - hr)^2 / hr^2 <= 1, in exact integers.
  int64_t a = 2 * (int64_t)u + 1 - wr, b = 2 * (int64_t)v + 1 - hr;
  return a * a * (int64_t)hr * hr + b * b * (int64_t)wr * wr <= (int64_t)wr * wr * (int64_t)hr * hr;
}

void add_noise(const sc_params& p, uint64_t purpose, int frame, uint8_t* img) {
  const int W = p.W, H = p.H, C = p.C;
#pragma omp parallel for schedule(static) if ((size_t)W * H > (1u << 18))
  for (int y = 0; y < H; ++y) {
    Rng r(p.seed, purpose, (uint64_t)frame, (uint64_t)y);
    Gauss g(r);
    uint8_t* row = img + (size_t)y * W * C;
    for (int i = 0; i < W * C; ++i)
      row[i] = clamp_u8(std::lround((double)row[i] + p.noise_sigma * g.next()));
  }
}

// Textures that do not change from frame to frame: the background and one
// texture per region (in region-local coordinates).
struct Textures {
  std::vector<uint8_t> bg;
  std::vector<std::vector<uint8_t>> reg;
};

void make_textures(const sc_params& p, Textures& t) {
  int bg_mean = -1;
  std::vector<Region> reg = layout(p, 0, &bg_mean);
  make_texture(p, P_BG_TEX, 0, p.W, p.H, bg_mean, t.bg);
  t.reg.resize(reg.size());
  for (size_t k = 0; k < reg.size(); ++k)
    make_texture(p, P_REG_TEX, (uint64_t)k, reg[k].wr, reg[k].hr, reg[k].mean, t.reg[k]);
}

int compose_frame(const sc_params& p, const Textures& tx, int32_t frame, uint8_t* left, uint8_t* right,
                  uint8_t* gt, uint8_t* occ, int16_t* rid);

}  // namespace

extern "C" {

// Makes frame `frame` of the scene. left/right: H*W*C bytes, HWC, pitch W*C.
// gt (u8, owner disparity per left pixel), occ (u8, 1 where the left pixel is
// not visible in the right image) and rid (i16, owning region or -1) are
// optional (NULL to skip). Returns 0, or -1 on bad parameters.
int sc_frame(const sc_params* pp, int32_t frame, uint8_t* left, uint8_t* right,
             uint8_t* gt, uint8_t* occ, int16_t* rid) {
  if (!pp || !left || !right) return -1;
  const sc_params& p = *pp;
  if (p.W < 1 || p.H < 1 || (p.C != 1 && p.C != 3) || p.dmax_regions < 0 || p.dmax_regions > 255)
    return -1;
  Textures tx;
  make_textures(p, tx);
  return compose_frame(p, tx, frame, left, right, gt, occ, rid);
}

}  // extern "C"

namespace {

// Fresh noise for pixels of the right image that no left pixel reaches: the
// same smoothed-uniform process as the textures, but with a counter-based
// source (a hash of (seed, frame, pixel, channel)) so single pixels can be
// drawn without making a whole noise image.
inline uint8_t hash_noise(const sc_params& p, int frame, int u, int v, int c) {
  uint64_t h = p.seed ^ (P_RIGHT * 0x9E3779B97F4A7C15ULL);
  h = mix64(h ^ ((uint64_t)frame * 0xD1B54A32D192ED03ULL + 1));
  h = mix64(h ^ (((uint64_t)v * (uint64_t)p.W + (uint64_t)u) * 0x8CB92BA72F3D8DD7ULL + (uint64_t)c));
  return (uint8_t)(h >> 56);
}

uint8_t fresh_value(const sc_params& p, int frame, int x, int y, int c, int mean) {
  const int W = p.W, H = p.H;
  int v;
  if (p.texture == 0) {
    int s = 0;
    for (int j = -1; j <= 1; ++j)
      for (int i = -1; i <= 1; ++i) s += hash_noise(p, frame, clampi(x + i, 0, W - 1), clampi(y + j, 0, H - 1), c);
    v = (s + 4) / 9;
  } else {
    double g[7], gs = 0;
    for (int k = -3; k <= 3; ++k) { g[k + 3] = std::exp(-0.5 * k * k); gs += g[k + 3]; }
    int64_t wt[7], ws = 0;
    for (int k = 0; k < 7; ++k) { wt[k] = (int64_t)std::llround(g[k] / gs * 65536.0); ws += wt[k]; }
    wt[3] += 65536 - ws;
    uint64_t s = 0;
    for (int j = -3; j <= 3; ++j) {
      uint64_t hsum = 0;
      for (int i = -3; i <= 3; ++i)
        hsum += (uint64_t)wt[i + 3] * hash_noise(p, frame, clampi(x + i, 0, W - 1), clampi(y + j, 0, H - 1), c);
      s += (uint64_t)wt[j + 3] * hsum;
    }
    v = (int)std::min<uint64_t>(255, (s + (1ULL << 31)) >> 32);
  }
  if (mean >= 0) {
    int d = v - 128;
    v = mean + (d >= 0 ? d / 2 : -((-d + 1) / 2));
  }
  return clamp_u8(v);
}

int compose_frame(const sc_params& p, const Textures& tx, int32_t frame, uint8_t* left, uint8_t* right,
                  uint8_t* gt, uint8_t* occ, int16_t* rid) {
  const int W = p.W, H = p.H, C = p.C;
  const size_t N = (size_t)W * H;
  int bg_mean = -1;
  std::vector<Region> reg = layout(p, frame, &bg_mean);
  std::memcpy(left, tx.bg.data(), N * C);
  std::vector<int16_t> zl(N, 0), own(N, -1);
  for (int k = 0; k < (int)reg.size(); ++k) {
    const Region& g = reg[k];
    const std::vector<uint8_t>& rt = tx.reg[(size_t)k];
    const int x0 = g.cx - g.wr / 2, y0 = g.cy - g.hr / 2;
    for (int v = 0; v < g.hr; ++v) {
      const int y = y0 + v;
      if (y < 0 || y >= H) continue;
      for (int u = 0; u < g.wr; ++u) {
        const int x = x0 + u;
        if (x < 0 || x >= W) continue;
        if (g.shape == 1 && !inside_ellipse(u, v, g.wr, g.hr)) continue;
        int d = g.disp;
        if (p.ramp && k == 0 && g.wr > 1) d += (16 * u + (g.wr - 1)) / (2 * (g.wr - 1));
        const size_t q = (size_t)y * W + x;
        if (d >= zl[q]) {
          std::memcpy(left + q * C, &rt[((size_t)v * g.wr + u) * C], C);
          zl[q] = (int16_t)d;
          own[q] = (int16_t)k;
        }
      }
    }
  }

  // Right image: a z-buffered forward warp of every left pixel to x - d on
  // the same row; pixels no left pixel reaches get fresh smoothed noise.
  std::vector<int16_t> zr(N, -1);
  std::vector<int32_t> src(N, -1);
#pragma omp parallel for schedule(static) if (N > (1u << 18))
  for (int y = 0; y < H; ++y) {
    for (int x = 0; x < W; ++x) {
      const size_t q = (size_t)y * W + x;
      const int d = zl[q];
      const int xr = x - d;
      if (xr < 0) continue;
      const size_t t = (size_t)y * W + xr;
      if (d >= zr[t]) {
        std::memcpy(right + t * C, left + q * C, C);
        zr[t] = (int16_t)d;
        src[t] = x;
      }
    }
  }
#pragma omp parallel for schedule(static) if (N > (1u << 18))
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const size_t t = (size_t)y * W + x;
      if (zr[t] >= 0) continue;
      for (int c = 0; c < C; ++c) right[t * C + c] = fresh_value(p, frame, x, y, c, bg_mean);
    }
  if (gt) for (size_t q = 0; q < N; ++q) gt[q] = (uint8_t)zl[q];
  if (occ) {
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        const size_t q = (size_t)y * W + x;
        const int xr = x - zl[q];
        occ[q] = (uint8_t)(xr < 0 || src[(size_t)y * W + xr] != x);
      }
  }
  if (rid) std::memcpy(rid, own.data(), N * sizeof(int16_t));
  if (p.noise_sigma > 0) {
    add_noise(p, P_NOISE_L, frame, left);
    add_noise(p, P_NOISE_R, frame, right);
  }
  return 0;
}

}  // namespace

extern "C" {

// Pixels near the scene's region outlines, the stand-in for a refined
// boundary set: the left and right image columns first, then pixels by
// ascending chessboard distance to the nearest outline pixel (a pixel whose
// region id differs from one of its 4-neighbours), ties broken by a seeded
// hash of the pixel index. Takes round(frac * W * H) pixels and writes them
// in ascending raster order. Returns the count, or -1 on bad arguments or
// when cap is too small.
int64_t sc_contour_list(const int16_t* rid, int32_t W, int32_t H, double frac,
                        uint64_t seed, uint32_t* out, int64_t cap) {
  if (!rid || !out || W < 1 || H < 1 || frac < 0.0 || frac > 1.0) return -1;
  const int64_t N = (int64_t)W * H;
  const int64_t want = std::min<int64_t>(N, std::llround(frac * (double)N));
  if (want > cap) return -1;
  const int32_t INF = 1 << 28;
  std::vector<int32_t> dist((size_t)N, INF);
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int16_t v = rid[(int64_t)y * W + x];
      bool edge = (x > 0 && rid[(int64_t)y * W + x - 1] != v) ||
                  (x + 1 < W && rid[(int64_t)y * W + x + 1] != v) ||
                  (y > 0 && rid[(int64_t)(y - 1) * W + x] != v) ||
                  (y + 1 < H && rid[(int64_t)(y + 1) * W + x] != v);
      if (edge) dist[(int64_t)y * W + x] = 0;
    }
  // Two-pass chessboard distance transform.
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int32_t& d = dist[(int64_t)y * W + x];
      if (x > 0) d = std::min(d, dist[(int64_t)y * W + x - 1] + 1);
      if (y > 0) {
        for (int i = -1; i <= 1; ++i)
          if (x + i >= 0 && x + i < W) d = std::min(d, dist[(int64_t)(y - 1) * W + x + i] + 1);
      }
    }
  for (int y = H - 1; y >= 0; --y)
    for (int x = W - 1; x >= 0; --x) {
      int32_t& d = dist[(int64_t)y * W + x];
      if (x + 1 < W) d = std::min(d, dist[(int64_t)y * W + x + 1] + 1);
      if (y + 1 < H) {
        for (int i = -1; i <= 1; ++i)
          if (x + i >= 0 && x + i < W) d = std::min(d, dist[(int64_t)(y + 1) * W + x + i] + 1);
      }
    }
  // Level 0: border columns; level 1 + dist otherwise (capped).
  const int32_t LCAP = 1 << 16;
  auto level = [&](int64_t q) -> int32_t {
    const int x = (int)(q % W);
    if (x == 0 || x == W - 1) return 0;
    return 1 + std::min(dist[(size_t)q], LCAP - 2);
  };
  std::vector<int64_t> hist((size_t)LCAP + 1, 0);
  for (int64_t q = 0; q < N; ++q) hist[(size_t)level(q)]++;
  int64_t acc = 0;
  int32_t cut = 0;
  while (cut <= LCAP && acc + hist[(size_t)cut] < want) { acc += hist[(size_t)cut]; ++cut; }
  const int64_t need = want - acc;  // how many to take from level `cut`
  std::vector<uint8_t> take((size_t)N, 0);
  std::vector<std::pair<uint64_t, int64_t>> tie;
  for (int64_t q = 0; q < N; ++q) {
    const int32_t l = level(q);
    if (l < cut) take[(size_t)q] = 1;
    else if (l == cut && need > 0) tie.emplace_back(mix64((uint64_t)q ^ seed), q);
  }
  if (need > 0) {
    std::nth_element(tie.begin(), tie.begin() + (need - 1), tie.end());
    for (int64_t i = 0; i < need; ++i) take[(size_t)tie[(size_t)i].second] = 1;
  }
  int64_t n = 0;
  for (int64_t q = 0; q < N; ++q)
    if (take[(size_t)q]) out[n++] = (uint32_t)q;
  return n;
}

// Makes frames [frame0, frame0 + nframes) of a video and, for each, a contour
// list with its own fraction fracs[i]. Frames are independent and are made in
// parallel. left/right: nframes * H*W*C bytes; lists: nframes * cap entries;
// counts[i] receives each list's length. Returns 0 or -1.
int sc_video(const sc_params* pp, int32_t frame0, int32_t nframes, uint8_t* left,
             uint8_t* right, const double* fracs, uint32_t* lists, int64_t cap,
             int64_t* counts) {
  if (!pp || nframes < 0) return -1;
  const sc_params& p = *pp;
  const size_t img = (size_t)p.W * p.H * p.C;
  const size_t N = (size_t)p.W * p.H;
  if (p.W < 1 || p.H < 1 || (p.C != 1 && p.C != 3) || p.dmax_regions < 0 || p.dmax_regions > 255)
    return -1;
  Textures tx;
  make_textures(p, tx);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int i = 0; i < nframes; ++i) {
    std::vector<int16_t> rid(N);
    int rc = compose_frame(p, tx, frame0 + i, left + img * i, right + img * i, nullptr, nullptr,
                           lists ? rid.data() : nullptr);
    if (rc != 0) { bad |= 1; continue; }
    if (lists) {
      int64_t n = sc_contour_list(rid.data(), p.W, p.H, fracs ? fracs[i] : 0.18,
                                  p.seed ^ (uint64_t)(frame0 + i), lists + (size_t)cap * i, cap);
      if (n < 0) bad |= 1;
      if (counts) counts[i] = n;
    }
  }
  return bad ? -1 : 0;
}

}  // extern "C"
