// Host-side check of the kernels' lane layouts (compiled with the system C++
// compiler against the same header the kernels include): every layout
// covers its tile's cells, chunks or columns exactly once, and in FP32 the
// words a half-wave of 32 lanes touches in the LDS tile buffers fall in 32
// distinct banks for the row pitches the kernels assert.
#include <cstdio>
#include <set>
#include <utility>
#include <vector>

#include "bq_layout.hpp"

using namespace bqk;

static int failures = 0;
#define CHECK(c, ...)                  \
  do {                                 \
    if (!(c)) {                        \
      std::printf("FAIL: " __VA_ARGS__); \
      std::printf("\n");               \
      ++failures;                      \
    }                                  \
  } while (0)

// every half-wave (32 consecutive entries) in distinct banks mod 32
static bool banks_distinct(const std::vector<int>& words) {
  for (size_t h = 0; h + 32 <= words.size(); h += 32) {
    std::set<int> b;
    for (size_t k = h; k < h + 32; ++k) b.insert(((words[k] % 32) + 32) % 32);
    if (b.size() != 32) return false;
  }
  return true;
}

template <typename T, int TY, int MX>
static void check_shape(const char* name, bool expect_conflict_free_solves_y) {
  constexpr int CPT = TX * TY / NT, PX = MX / 8, NCX = TX / MX;
  constexpr bool f32 = sizeof(T) == 4;
  // pitches with the residues the kernels assert (radius-2 tile, result rows, corners)
  const int LW = 32 * 3 + PITCH_MOD_TILE, AXP = 32 * 2 + PITCH_MOD_ROWS, CP = 32 * 2 + PITCH_MOD_CORNERS;
  // cells of the per-cell phases
  std::set<std::pair<int, int>> cells;
  std::vector<int> w_tile, w_rows, w_corner;
  for (int t = 0; t < NT; ++t) {
    int vr = -1, vc = -1;
    cell_of<T, CPT>(t, vr, vc);
    CHECK(vr >= 0 && vr < TY && vc >= 0 && vc + CPT <= TX, "%s: thread %d cells (%d, %d) outside the tile", name, t,
          vr, vc);
    for (int k = 0; k < CPT; ++k) cells.insert({vr, vc + k});
    w_tile.push_back(vr * LW + vc);
    w_rows.push_back(vr * AXP + vc);
    w_corner.push_back(vr * CP + vc);
  }
  CHECK((int)cells.size() == TX * TY, "%s: the threads cover %zu of %d cells", name, cells.size(), TX * TY);
  if (f32) {
    CHECK(banks_distinct(w_tile), "%s: per-cell reads of the radius-2 tiles conflict", name);
    CHECK(banks_distinct(w_rows), "%s: per-cell reads of the result rows conflict", name);
    CHECK(banks_distinct(w_corner), "%s: per-cell reads of the corner tile conflict", name);
  }
  // x-chunk lane groups: PX parts of 8 columns
  std::set<std::pair<int, int>> chunks;
  std::vector<int> w_xs, w_xu;
  for (int qq = 0; qq < TY * NCX; ++qq) {
    int r = -1, qc = -1;
    xchunk_of<T, TY, NCX, PX>(qq, r, qc);
    CHECK(r >= 0 && r < TY && qc >= 0 && qc < NCX, "%s: group %d at row %d chunk %d", name, qq, r, qc);
    chunks.insert({r, qc});
    for (int p = 0; p < PX; ++p) {
      w_xs.push_back(r * LW + qc * MX + 8 * p);
      w_xu.push_back(r * AXP + qc * MX + 8 * p);
    }
  }
  CHECK((int)chunks.size() == TY * NCX, "%s: the groups cover %zu of %d x-chunks", name, chunks.size(), TY * NCX);
  if (f32) {
    CHECK(banks_distinct(w_xs), "%s: x-chunk depth reads conflict", name);
    CHECK(banks_distinct(w_xu), "%s: x-chunk right-hand-side reads conflict", name);
  }
  // y-chunk lane pairs: two parts of TY / 2 rows
  std::set<int> cols;
  std::vector<int> w_ys, w_yv;
  for (int g = 0; g < TX; ++g) {
    const int c = ycol_of<T, TY>(g);
    CHECK(c >= 0 && c < TX, "%s: pair %d at column %d", name, g, c);
    cols.insert(c);
    for (int p = 0; p < 2; ++p) {
      w_ys.push_back(c + (TY / 2) * p * LW);
      w_yv.push_back(c + (TY / 2) * p * AXP);
    }
  }
  CHECK((int)cols.size() == TX, "%s: the pairs cover %zu of %d columns", name, cols.size(), TX);
  if (f32 && expect_conflict_free_solves_y) {
    CHECK(banks_distinct(w_ys), "%s: y-chunk depth reads conflict", name);
    CHECK(banks_distinct(w_yv), "%s: y-chunk right-hand-side reads conflict", name);
  }
  std::printf("%s checked\n", name);
}

// pair staging of an NR x 2 NPR tile: every cell staged, and owned by
// exactly one thread, whose row is its own (not a repeat)
template <int NPR, int NR>
static void check_staging(const char* name) {
  using S = PairStaging<NPR, NR>;
  std::vector<int> staged(NR * 2 * NPR, 0), owned(NR * 2 * NPR, 0);
  for (int t = 0; t < NT; ++t)
    for (int k = 0; k < S::K; ++k) {
      const int r = S::row(t, k), c = S::col(t);
      CHECK(r >= 0 && r < NR && c >= 0 && c + 1 < 2 * NPR, "%s: thread %d round %d at (%d, %d)", name, t, k, r, c);
      if (!(r >= 0 && r < NR && c >= 0 && c + 1 < 2 * NPR)) continue;
      for (int u = 0; u < 2; ++u) {
        ++staged[r * 2 * NPR + c + u];
        if (S::owns(t, k)) ++owned[r * 2 * NPR + c + u];
      }
      if (S::owns(t, k)) CHECK(r == S::r0(t) + S::RG * k, "%s: thread %d owns a repeated row", name, t);
    }
  for (int e = 0; e < NR * 2 * NPR; ++e) {
    CHECK(staged[e] >= 1, "%s: cell %d never staged", name, e);
    CHECK(owned[e] == 1, "%s: cell %d owned by %d threads", name, e, owned[e]);
  }
  std::printf("%s staging checked\n", name);
}

int main() {
  // the stencil kernel's radius-2 rows, radius-1 rows and corner rows, the
  // finalize kernel's corner rows, for tile heights 16, 8 and 4
  check_staging<(TX + 4) / 2, 16 + 4>("radius-2 rows, TY 16");
  check_staging<(TX + 4) / 2, 8 + 4>("radius-2 rows, TY 8");
  check_staging<(TX + 4) / 2, 4 + 4>("radius-2 rows, TY 4");
  check_staging<(TX + 4) / 2, 16 + 2>("radius-1 rows, TY 16");
  check_staging<(TX + 4) / 2, 8 + 2>("radius-1 rows, TY 8");
  check_staging<(TX + 4) / 2, 4 + 2>("radius-1 rows, TY 4");
  check_staging<(TX + 6) / 2, 16 + 5>("corner rows, TY 16");
  check_staging<(TX + 6) / 2, 8 + 5>("corner rows, TY 8");
  check_staging<(TX + 6) / 2, 4 + 5>("corner rows, TY 4");
  check_staging<(TX + 4) / 2, 16 + 3>("finalize corner rows, TY 16");
  check_staging<(TX + 4) / 2, 8 + 3>("finalize corner rows, TY 8");
  check_staging<(TX + 4) / 2, 4 + 3>("finalize corner rows, TY 4");
  check_shape<float, 16, 16>("fp32 16x16", true);
  check_shape<float, 16, 32>("fp32 16x32", true);
  check_shape<float, 8, 16>("fp32 8x16", false);
  check_shape<float, 8, 32>("fp32 8x32", false);
  check_shape<double, 8, 16>("fp64 8x16", false);
  check_shape<double, 8, 32>("fp64 8x32", false);
  check_shape<double, 4, 16>("fp64 4x16", false);
  if (failures) std::printf("%d failures\n", failures);
  return failures ? 1 : 0;
}
