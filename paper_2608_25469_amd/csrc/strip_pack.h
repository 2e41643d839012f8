// Order of one bucket's strips in the grouped strip launch (host code, no
// HIP dependency).
//
// A bucket holds the 16-column strips of problems that share m, problem by
// problem; a wavefront solves four consecutive strips, one per DPP row.
// The strips of one problem in one wavefront read L through the same loads
// (equal addresses in one instruction), while a problem split over two
// wavefronts has its L read twice.  So each problem's first 4 floor(k / 4)
// strips fill whole wavefronts of their own; the remainders (k mod 4 strips,
// 1..3) fill wavefronts whose sizes add up to four (3 + 1; 2 + 2; 2 + 1 + 1;
// 1 + 1 + 1 + 1); the remainders left over follow one another and may
// straddle wavefronts.  No more wavefronts than packing the strips in
// problem order, and every strip appears exactly once.

#pragma once

#include <cstddef>
#include <vector>

namespace hsma {

struct StripSpan {
    int first;  // index of the problem's first strip in the bucket
    int k;      // its strip count (>= 1)
};

// Appends the strips of `v` (problems described by `spans`) to `out` in
// wavefront order.  The caller pads the bucket's last wavefront.
template <typename Item>
void pack_bucket(const std::vector<Item> &v, const std::vector<StripSpan> &spans,
                 std::vector<Item> &out) {
    std::vector<int> by_r[4];  // problems by remainder size 1..3
    for (int i = 0; i < (int)spans.size(); ++i) {
        const int full = spans[i].k / 4 * 4;
        for (int j = 0; j < full; ++j) out.push_back(v[spans[i].first + j]);
        if (spans[i].k > full) by_r[spans[i].k - full].push_back(i);
    }
    auto emit = [&](int i) {
        for (int j = spans[i].k / 4 * 4; j < spans[i].k; ++j) out.push_back(v[spans[i].first + j]);
    };
    const std::vector<int> &r3 = by_r[3], &r2 = by_r[2], &r1 = by_r[1];
    size_t i3 = 0, i2 = 0, i1 = 0;
    for (; i3 < r3.size() && i1 < r1.size(); ++i3, ++i1) {
        emit(r3[i3]);
        emit(r1[i1]);
    }
    for (; i2 + 1 < r2.size(); i2 += 2) {
        emit(r2[i2]);
        emit(r2[i2 + 1]);
    }
    if (i2 < r2.size() && i1 + 1 < r1.size()) {
        emit(r2[i2++]);
        emit(r1[i1++]);
        emit(r1[i1++]);
    }
    for (; i1 + 3 < r1.size(); i1 += 4)
        for (int j = 0; j < 4; ++j) emit(r1[i1 + j]);
    for (; i3 < r3.size(); ++i3) emit(r3[i3]);
    for (; i2 < r2.size(); ++i2) emit(r2[i2]);
    for (; i1 < r1.size(); ++i1) emit(r1[i1]);
}

}  // namespace hsma
