// HSS handle shared by the construction, matvec and ULV units.
#pragma once
#include "common.h"

struct hss_s {
    long N = 0;
    int leaf = 0, Lh = 0;
    // rank[l][j] and effective leaf size m[l][j] for 1 <= l <= Lh (index 0 unused; m[0][0] = root size)
    std::vector<std::vector<int>> rank, m;
    // U_(l,j) lives in an m x m column-major slot (only the first r columns are used):
    // element offset uoff[l][j] inside Ubuf[l]
    std::vector<std::vector<size_t>> uoff;
    std::vector<fio::DevBuf *> Ubuf;
    // B_(l,j) = B_{a2,a1} (r_a2 x r_a1, column-major) packed in Bbuf at boff[l][j], 0 <= l < Lh
    std::vector<std::vector<size_t>> boff;
    fio::DevBuf Bbuf;
    // leaf diagonal blocks, leaf x leaf each, contiguous
    fio::DevBuf Dbuf;
    double gain = 0.0;
    std::vector<int> samples;   // s_l used by the construction (the last draw of a level)
    std::vector<int> drawn;     // sample columns drawn per level (more than s_l after a redraw)
    bool rank_capped = false;
    ~hss_s() {
        for (auto *b : Ubuf) delete b;
    }
    int nodes(int l) const { return 1 << l; }
    const double2 *U(int l, int j) const { return Ubuf[l]->as<double2>() + uoff[l][j]; }
    double2 *U(int l, int j) { return Ubuf[l]->as<double2>() + uoff[l][j]; }
    const double2 *B(int l, int j) const { return Bbuf.as<double2>() + boff[l][j]; }
    double2 *B(int l, int j) { return Bbuf.as<double2>() + boff[l][j]; }
    double2 *D(int j) { return Dbuf.as<double2>() + (size_t)j * leaf * leaf; }
    const double2 *D(int j) const { return Dbuf.as<double2>() + (size_t)j * leaf * leaf; }
};

namespace fio {
// sets m[][] and uoff from rank[][] (levels Lh..1) and allocates the U slots of level l
void hss_layout_level(hss_s *h, int l);
void hss_layout_B(hss_s *h);
}  // namespace fio
