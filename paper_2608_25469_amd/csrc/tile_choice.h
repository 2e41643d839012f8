// Tile shapes of the FP64 product (host code, no HIP dependency).
//
// A workgroup stages its A and B tiles through a two-stage LDS ring of
// BK-deep slices; the ring's size sets how many workgroups a CU holds (160 KB
// of LDS, at most three).  For a lower-triangular C only the tiles on or
// below the diagonal run, and each runs the whole K, so a launch takes about
// ceil(non-empty tiles / resident slots) rounds of one tile's time;
// lower_tile_shape picks the shape with the fewest rounds times tile area,
// weighted by the shape's relative throughput (narrower tiles reuse less of
// what they stage).

#pragma once

#include <algorithm>
#include <cstdint>

namespace hsma {

constexpr int kTileBK = 16;

constexpr int tile_lds_bytes(int bm, int bn) { return 2 * (kTileBK * (bm + 4) + bn * (kTileBK + 1)) * 8; }

constexpr int tile_occupancy(int bm, int bn) {
    return (160 * 1024 / tile_lds_bytes(bm, bn)) >= 3 ? 3 : ((160 * 1024 / tile_lds_bytes(bm, bn)) >= 2 ? 2 : 1);
}

struct TileShape {
    int bm, bn;
    double eff;  // throughput relative to 128 x 128
};
// The weights of the two smallest shapes are extrapolated from the others by
// operand reuse (bm bn / (bm + bn) per staged element: 64, 43, 32, 21, 16).
constexpr int kNumLowerShapes = 5;
constexpr TileShape kLowerShapes[kNumLowerShapes] = {
    {128, 128, 1.0}, {128, 64, 0.85}, {64, 64, 0.7}, {64, 32, 0.5}, {32, 32, 0.35}};

// Tiles of an M x N (real-view) lower-triangular C that hold an element on
// or below the diagonal; complex C has two real-view rows per row.
inline int64_t lower_tiles(int64_t M, int64_t N, bool cx, int bm, int bn) {
    const int64_t tm_n = (M + bm - 1) / bm, tn_n = (N + bn - 1) / bn;
    int64_t tiles = 0;
    for (int64_t tm = 0; tm < tm_n; ++tm) {
        const int64_t last = cx ? (tm * bm + bm - 1) / 2 : tm * bm + bm - 1;
        tiles += std::min<int64_t>(tn_n, last / bn + 1);
    }
    return tiles;
}

// Index into kLowerShapes for `count` products of that size on `cus` CUs.
inline int lower_tile_shape(int64_t M, int64_t N, bool cx, int count, int64_t cus) {
    int best = 0;
    double best_cost = 0.0;
    for (int k = 0; k < kNumLowerShapes; ++k) {
        const TileShape &t = kLowerShapes[k];
        const int64_t tiles = lower_tiles(M, N, cx, t.bm, t.bn) * count;
        const int64_t slots = (int64_t)tile_occupancy(t.bm, t.bn) * cus;
        const double cost = (double)((tiles + slots - 1) / slots) * t.bm * t.bn / t.eff;
        if (k == 0 || cost < best_cost) {
            best = k;
            best_cost = cost;
        }
    }
    return best;
}

}  // namespace hsma
