// Tile geometry and the lanes' layouts over a tile, shared by the stencil
// and finalize kernels.  Plain integer constexpr functions (callable from
// device code and from host code, where a CPU test checks that every layout
// covers its tile exactly once and, in FP32, touches 32 distinct LDS banks
// per half-wave).
#pragma once

namespace bqk {

constexpr int TX = 64;      // tile width (cells)
constexpr int NT = 256;     // threads per tile block

// Row pitches (words, mod 32) of the LDS tile buffers that the layouts
// below assume: the radius-2 tiles and the finalize kernel's depth tile 5,
// the per-cell result rows 1, the corner tile 9.
constexpr int PITCH_MOD_TILE = 5, PITCH_MOD_ROWS = 1, PITCH_MOD_CORNERS = 9;

// Lane layouts of the per-cell phases and the chunk solves.  LDS serves a
// wave in two halves of 32 lanes over 32 banks of 4 bytes, so a half-wave's
// 32 words are conflict-free when they fall in distinct banks mod 32.  The
// tile buffers have odd row pitches (5 or 1 mod 32 words), which the
// layouts below rely on; FP64 keeps the plain row-major layouts.
//
// Cells of thread t: CPT consecutive columns vc .. vc+CPT-1 of row vr.  In
// FP32 each half-wave takes CPT rows of 32 columns (32/CPT lanes per row),
// so its CPT-strided words cover every bank once.
template <typename T, int CPT>
constexpr void cell_of(int t, int& vr, int& vc) {
  if constexpr (sizeof(T) == 4 && CPT > 1) {
    constexpr int LS = 32 / CPT;                   // lanes per 32-column row segment
    const int w = t >> 6, half = (t >> 5) & 1, h = t & 31;
    vr = CPT * w + h / LS;
    vc = 32 * half + CPT * (h % LS);
  } else {
    constexpr int SPR = TX / CPT;
    vr = t / SPR;
    vc = (t - vr * SPR) * CPT;
  }
}
// Row r and chunk qc of x-chunk lane group qq (PX lanes, parts of 8
// columns): in FP32 each half-wave's 32 / PX groups take 8 rows of 4 / PX
// chunks, so the parts' first columns (8 apart) fall in distinct banks.
template <typename T, int TY, int NCX, int PX>
constexpr void xchunk_of(int qq, int& r, int& qc) {
  if constexpr (sizeof(T) == 4 && TY % 8 == 0 && (32 / PX) % 8 == 0) {
    constexpr int HC = 32 / PX, QH = HC / 8, RB = TY / 8;
    const int hw = qq / HC, i = qq - hw * HC;
    r = 8 * (hw % RB) + (i & 7);
    qc = QH * (hw / RB) + (i >> 3);
  } else {
    r = qq / NCX;
    qc = qq - r * NCX;
  }
}
// Tile column of y-chunk lane pair g (parts of TY / 2 rows): in FP32 with
// 16-row tiles each half-wave's 16 pairs take two runs of 8 columns 16
// apart, so the two parts (8 rows apart: 8 mod 32 words) fall in distinct
// banks.
template <typename T, int TY>
constexpr int ycol_of(int g) {
  if constexpr (sizeof(T) == 4 && TY == 16) {
    const int hw = g >> 4, i = g & 15;
    return 32 * (hw >> 1) + 8 * (hw & 1) + 16 * (i >> 3) + (i & 7);
  }
  return g;
}

// Staging of an LDS tile of NR rows by 2 NPR columns in pairs of cells by
// the NT threads of a block: thread t loads the pair of columns col(t) =
// 2 (t mod NPR) of rows row(t, k) = r0(t) + RG k, k = 0 .. K - 1, with RG =
// NT / NPR whole rows per round.  Threads past the last whole row repeat
// row RG - 1, and rows past the tile repeat its last row, so every round is
// branch-free (the repeats store the same values again); owns(t, k) marks
// the one thread of each cell, for the passes that update a cell in place.
template <int NPR, int NR>
struct PairStaging {
  static constexpr int RG = NT / NPR, K = (NR + RG - 1) / RG;
  static_assert(RG >= 1, "a row of pairs must fit the block");
  static constexpr int r0(int t) { return t / NPR < RG - 1 ? t / NPR : RG - 1; }
  static constexpr int col(int t) { return 2 * (t - (t / NPR) * NPR); }
  static constexpr int row(int t, int k) {
    return k < K - 1 ? r0(t) + RG * k : (r0(t) + RG * k < NR - 1 ? r0(t) + RG * k : NR - 1);
  }
  static constexpr bool owns(int t, int k) { return t < NPR * RG && r0(t) + RG * k < NR; }
};

}  // namespace bqk
