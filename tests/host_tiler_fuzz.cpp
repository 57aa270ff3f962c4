// Host tiler under AddressSanitizer and UndefinedBehaviorSanitizer: random
// bitmaps of every size from 1 to 19 per axis (ragged tiles), every periodic
// combination, all-fluid, all-solid and random fills; the fluid count must
// equal the masks' popcount, failures must leave no tiles behind.  Built and
// run by test_host_sanitizers.py with g++ (host code only).
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "lbm.h"
int main() {
    unsigned seed = 1;
    auto rnd = [&]() { seed = seed * 1103515245u + 12345u; return (seed >> 16) & 0x7fff; };
    int fails = 0;
    for (int it = 0; it < 400; ++it) {
        int nx = 1 + rnd() % 19, ny = 1 + rnd() % 19, nz = 1 + rnd() % 19;
        int per = rnd() % 8;
        std::vector<uint8_t> s((size_t)nx * ny * nz);
        int mode = rnd() % 4;
        for (auto &v : s) v = mode == 0 ? 0 : mode == 1 ? 1 : (rnd() % 100) < (mode == 2 ? 30 : 90);
        lbm_tiles *t = nullptr;
        int rc = lbm_build_tiles(s.data(), nx, ny, nz, per, &t);
        if (rc == 0) {
            long long fl = 0;
            for (int i = 0; i < t->n_tiles; ++i) fl += __builtin_popcountll(t->fluid_mask[i]);
            if (fl != t->n_fluid) { std::printf("n_fluid mismatch\n"); ++fails; }
            lbm_tiles_free(t);
        } else if (t) { std::printf("tiles set on failure\n"); ++fails; }
    }
    lbm_tiles *t = nullptr;
    if (lbm_build_tiles(nullptr, 4, 4, 4, 0, &t) == 0) ++fails;
    uint8_t one = 0;
    if (lbm_build_tiles(&one, 0, 4, 4, 0, &t) == 0) { lbm_tiles_free(t); }
    std::printf("done fails=%d\n", fails);
    return fails;
}
