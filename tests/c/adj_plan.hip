// Host check of the adjoint's wave plan (adj_plan / adj_segment): for many
// grid shapes and CU counts every (strip, row) belongs to exactly one wave,
// segments are non-empty and in range, lengths differ by at most one row,
// and with two waves per SIMD no SIMD holds two long segments while a short
// one remains in either pairing of a block's waves.
#include <cstdio>
#include <vector>

#include "adjoint2d.hpp"

using namespace mp;

template <int WPB>
static int check(int nx, int ny, int cus) {
    AdjGeom g{};
    g.nx = nx;
    g.ny = ny;
    adj_plan(g, cus * WPB);
    const int nb = adj_blocks<WPB>(g);
    std::vector<int> cov((size_t)g.ntx * ny, 0);
    long long nlong_a = 0, nlong_b = 0;
    for (int b = 0; b < nb; ++b) {
        int len[8] = {0};
        for (int w = 0; w < WPB; ++w) {
            int tx, m0, m1;
            adj_segment<WPB>(g, b * WPB + w, tx, m0, m1);
            if (tx >= g.ntx) continue;
            if (m0 < 0 || m1 > ny || m1 <= m0) return 1;
            if (m1 - m0 != g.len && m1 - m0 != g.len + 1) return 2;
            for (int m = m0; m < m1; ++m) cov[(size_t)tx * ny + m]++;
            len[w] = m1 - m0;
        }
        if (WPB == 8 && g.nlong <= g.pw / 2 - 4) {
            // both pairings (w, w+4) and (2i, 2i+1): at most one long segment per pair
            for (int i = 0; i < 4; ++i) {
                if (len[i] > g.len && len[i + 4] > g.len) nlong_a++;
                if (len[2 * i] > g.len && len[2 * i + 1] > g.len) nlong_b++;
            }
        }
    }
    for (int c : cov)
        if (c != 1) return 3;
    if (nlong_a || nlong_b) return 4;
    return 0;
}

int main() {
    const int sizes[][2] = {{512, 512}, {64, 64}, {1, 1}, {1, 40}, {40, 1}, {3, 2}, {62, 62}, {63, 2049},
                            {130, 1000}, {4096, 4096}, {5000, 17}, {200000, 3}, {777, 333}};
    for (const auto& s : sizes)
        for (int cus : {256, 80, 7, 1}) {
            int e = check<8>(s[0], s[1], cus);
            if (!e) e = check<4>(s[0], s[1], cus);
            if (e) {
                std::printf("fail %d at %d x %d, %d CUs\n", e, s[0], s[1], cus);
                return 1;
            }
        }
    std::printf("ok\n");
    return 0;
}
