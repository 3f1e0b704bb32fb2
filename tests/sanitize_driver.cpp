// Host-side driver for the sanitizer test (tests/test_sanitizers.py): calls
// the oracle, the scene generator and the library's host-only paths
// (validation, workspace sizing, plans, tuning-cache load/save) on small
// inputs. Built with AddressSanitizer and UndefinedBehaviorSanitizer.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

extern "C" {
struct sc_params {
  int32_t W, H, C, n_regions, dmax_regions, texture, mean_shift, ramp, motion, drift;
  double noise_sigma;
  uint64_t seed;
};
int sc_frame(const sc_params*, int32_t, uint8_t*, uint8_t*, uint8_t*, uint8_t*, int16_t*);
int64_t sc_contour_list(const int16_t*, int32_t, int32_t, double, uint64_t, uint32_t*, int64_t);
int64_t oracle_boundaries(const uint8_t*, int32_t, int32_t, int32_t, int64_t, int32_t, int32_t, int64_t, double,
                          uint64_t, uint32_t*, int64_t, uint8_t*);
int oracle_sad(const uint8_t*, const uint8_t*, int32_t, int32_t, int32_t, int64_t, const uint32_t*, int64_t, int32_t,
               int32_t, uint8_t*, uint32_t*, int32_t);
int oracle_sad_sat(const uint8_t*, const uint8_t*, int32_t, int32_t, int32_t, int64_t, const uint32_t*, int64_t,
                   int32_t, int32_t, uint8_t*, uint32_t*);
void oracle_reconstruct(const uint32_t*, const uint8_t*, int64_t, int32_t, int32_t, int32_t, uint8_t*);
void oracle_blur(const uint8_t*, int32_t, int32_t, int32_t, int64_t, const uint8_t*, const int32_t*, int32_t, double,
                 float*);
#ifdef WITH_LIB
typedef struct { const uint8_t *left, *right; int32_t W, H, C; int64_t pitch_bytes; const uint32_t* boundary_idx;
                 int64_t n; int32_t block, dmax; uint8_t* out_disp; uint32_t* out_cost; } sbs_frame;
typedef struct { int32_t cols_per_lane, chunk, tile_rows, waves_per_cu; } sbs_plan;
int sbs_sad_disparity(const uint8_t*, const uint8_t*, int32_t, int32_t, int32_t, int64_t, const uint32_t*, int64_t,
                      int32_t, int32_t, uint8_t*, uint32_t*, void*, size_t, void*);
size_t sbs_workspace_bytes(const sbs_frame*, int32_t);
int sbs_set_plan(const sbs_plan*);
int sbs_get_plan(const sbs_frame*, sbs_plan*);
int sbs_load_tuning(const char*);
const char* sbs_last_error(void);
#endif
}

int main(int argc, char** argv) {
  const int W = 96, H = 64;
  sc_params p{W, H, 3, 5, 12, 0, 1, 1, 0, 0, 1.5, 42};
  std::vector<uint8_t> L(W * H * 3), R(W * H * 3), gt(W * H), occ(W * H);
  std::vector<int16_t> rid(W * H);
  if (sc_frame(&p, 0, L.data(), R.data(), gt.data(), occ.data(), rid.data()) != 0) return 2;
  std::vector<uint32_t> idx(W * H);
  int64_t n = sc_contour_list(rid.data(), W, H, 0.2, 7, idx.data(), (int64_t)idx.size());
  if (n <= 0) return 3;
  std::vector<uint32_t> fl(W * H);
  std::vector<uint8_t> rm(W * H);
  if (oracle_boundaries(L.data(), W, H, 3, W * 3, 4, 0, 50, 0.18, 1, fl.data(), (int64_t)fl.size(), rm.data()) < 0) return 4;
  if (oracle_boundaries(L.data(), W, H, 3, W * 3, 10, 1, 0, -1.0, 1, fl.data(), (int64_t)fl.size(), rm.data()) < 0) return 5;
  std::vector<uint8_t> d1(n), d2(n);
  std::vector<uint32_t> c1(n), c2(n);
  oracle_sad(L.data(), R.data(), W, H, 3, W * 3, idx.data(), n, 7, 15, d1.data(), c1.data(), 2);
  oracle_sad_sat(L.data(), R.data(), W, H, 3, W * 3, idx.data(), n, 7, 15, d2.data(), c2.data());
  if (std::memcmp(d1.data(), d2.data(), n) || std::memcmp(c1.data(), c2.data(), n * 4)) return 6;
  std::vector<uint8_t> dense(W * H);
  oracle_reconstruct(idx.data(), d1.data(), n, W, H, 1, dense.data());
  std::vector<float> blurred(W * H * 3);
  const int32_t ranges[2] = {3, 8};
  oracle_blur(L.data(), W, H, 3, W * 3, dense.data(), ranges, 1, 1.2, blurred.data());
#ifdef WITH_LIB
  // Host-only library paths: validation, sizing, plans, tuning cache.
  if (sbs_sad_disparity(L.data(), R.data(), 0, H, 3, W * 3, idx.data(), n, 7, 15, d1.data(), nullptr, nullptr, 0,
                        nullptr) != 1) return 7;
  if (std::strlen(sbs_last_error()) == 0) return 8;
  sbs_frame f{L.data(), R.data(), W, H, 3, W * 3, idx.data(), n, 7, 15, d1.data(), nullptr};
  if (sbs_workspace_bytes(&f, 1) == 0) return 9;
  sbs_plan pl{0, 8, 32, 4}, got{};
  if (sbs_set_plan(&pl) != 0 || sbs_get_plan(&f, &got) != 0 || got.tile_rows != 32) return 10;
  sbs_plan none{0, 0, 0, 0};
  sbs_set_plan(&none);
  if (argc > 1 && sbs_load_tuning(argv[1]) != 0) return 11;
#endif
  std::printf("sanitize driver ok\n");
  return 0;
}
