// Host check of the lower-triangular product's tile shape choice
// (csrc/tile_choice.h): the count of non-empty tiles against a brute force
// over elements, and the shapes chosen for three sizes worked out by hand
// (256 CUs): the top-level updates of a complex n = 8192 and a real
// n = 16384 Cholesky (128 x 64: three and six rounds against three and five
// of twice the area), and a real 3968 x 3968 product (128 x 128: one round of
// 496 tiles, where 128 x 64 would need two).
#include <cstdio>

#include "tile_choice.h"

using namespace hsma;

static long long brute(long long M, long long N, bool cx, int bm, int bn) {
    long long tiles = 0;
    for (long long r0 = 0; r0 < M; r0 += bm)
        for (long long c0 = 0; c0 < N; c0 += bn) {
            bool any = false;
            for (long long r = r0; r < r0 + bm && r < M && !any; ++r)
                for (long long c = c0; c < c0 + bn && c < N; ++c)
                    if (c <= (cx ? r / 2 : r)) {
                        any = true;
                        break;
                    }
            tiles += any;
        }
    return tiles;
}

int main() {
    int bad = 0;
    const long long sizes[][2] = {{1, 1}, {64, 64}, {130, 70}, {256, 512}, {600, 300}, {1000, 999}, {2048, 1024}};
    for (const auto &sz : sizes)
        for (int cx = 0; cx < 2; ++cx)
            for (const TileShape &t : kLowerShapes) {
                const long long a = lower_tiles(sz[0], sz[1], cx, t.bm, t.bn), b = brute(sz[0], sz[1], cx, t.bm, t.bn);
                if (a != b) {
                    std::printf("tiles M=%lld N=%lld cx=%d %dx%d: %lld, brute force %lld\n", sz[0], sz[1], cx, t.bm, t.bn, a, b);
                    ++bad;
                }
            }
    struct Case {
        long long M, N;
        bool cx;
        int want;
    } cases[] = {{8192, 4096, true, 1}, {8192, 8192, false, 1}, {3968, 3968, false, 0},
                 // 4096 x 4096 real: three rounds of 64 x 64 tiles beat six of 64 x 32
                 {4096, 4096, false, 2},
                 // one round for every shape: the smallest tile (the most CUs busy)
                 {256, 128, true, 4}, {128, 128, false, 4}};
    for (const Case &c : cases) {
        const int got = lower_tile_shape(c.M, c.N, c.cx, 1, 256);
        if (got != c.want) {
            std::printf("shape M=%lld N=%lld cx=%d: %d, expected %d\n", c.M, c.N, (int)c.cx, got, c.want);
            ++bad;
        }
    }
    if (tile_occupancy(128, 128) != 2 || tile_occupancy(128, 64) != 3 || tile_occupancy(64, 64) != 3 ||
        tile_occupancy(64, 32) != 3 || tile_occupancy(32, 32) != 3) {
        std::printf("occupancy %d %d %d\n", tile_occupancy(128, 128), tile_occupancy(128, 64), tile_occupancy(64, 64));
        ++bad;
    }
    if (bad) return 1;
    std::printf("tile choice ok\n");
    return 0;
}
