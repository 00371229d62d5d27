// Host-side tile plans, map tables, box and matrix-core tables for 400 random
// NBB fractals (s 2..5, any k, r <= 8, every tile level, both team sizes),
// built under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py.
#include <algorithm>
#include <cstdio>
#include <random>
#include <string>
#include <vector>
#include "plan.hpp"
using namespace nbb;
int main() {
    std::mt19937 rng(12345);
    int plans = 0, maps = 0;
    for (int it = 0; it < 400; ++it) {
        uint32_t s = 2 + rng() % 4;            // 2..5
        uint32_t k = 1 + rng() % (s * s);
        std::vector<int> cells(s * s);
        for (uint32_t i = 0; i < s * s; ++i) cells[i] = int(i);
        std::shuffle(cells.begin(), cells.end(), rng);
        std::vector<int32_t> off;
        for (uint32_t j = 0; j < k; ++j) { off.push_back(cells[j] % s); off.push_back(cells[j] / s); }
        uint32_t r = rng() % 9;
        Fractal f; std::string msg;
        if (validate_fractal(k, s, off.data(), r, &f, &msg)) continue;
        double cellsr = 1; for (uint32_t i = 0; i < r; ++i) cellsr *= k;
        if (cellsr > 2e6) continue;
        MapTables mt; build_map_tables(f, &mt); ++maps;
        BoxTables bt; build_box_tables(f, &bt);
        MfmaTables ft; build_mfma_tables(f, &ft);
        if (!tiled_supported(f)) continue;
        for (uint32_t m = 1; m <= r; ++m)
            for (uint32_t team : {256u, 64u}) {
                TilePlan p;
                if (build_tile_plan(f, m, &p, &msg, team)) ++plans;
            }
        (void)auto_tile_level(f);
    }
    std::printf("maps %d plans %d\n", maps, plans);
    return 0;
}
