// Host check of the pair-slot index used by the fixed-order backward: for
// random pixel boxes (one column interval, or two when the box wraps past the
// last column, merged when they meet in tile columns) and every tile shape,
// span_index must invert the emit order of tile_span -- row by row, first
// interval then second -- exactly.  Prints the count of mismatches; exit 1 on any.
#include "../../paper_2503_17491_amd/csrc/slr_internal.h"

#include <cstdio>
#include <random>

int main()
{
    std::mt19937 g(12345);
    const int shapes[4][2] = {{16, 16}, {8, 32}, {32, 8}, {4, 64}};
    long bad = 0, total = 0;
    for (int it = 0; it < 40000; ++it) {
        const int th = shapes[it % 4][0], tw = shapes[it % 4][1];
        const int W = 64 + (int)(g() % 2000), H = 16 + (int)(g() % 128);
        slr::PixBox b{};
        b.r0 = (int16_t)(g() % H);
        b.r1 = (int16_t)(b.r0 + g() % (H - b.r0));
        b.c0 = (int16_t)(g() % W);
        b.c1 = (int16_t)(b.c0 + g() % (W - b.c0));
        b.c2 = -1;
        b.c3 = -1;
        if (g() % 2) {   // wrapped: [c0, W - 1] and [0, c3]
            b.c1 = (int16_t)(W - 1);
            b.c2 = 0;
            b.c3 = (int16_t)(g() % (b.c0 + 1));
        }
        const slr::TileSpan sp = slr::tile_span(b, th, tw);
        const int rows = b.r1 / th - b.r0 / th + 1;
        for (int j = 0; j < rows * sp.len; ++j) {
            const int dy = j / sp.len, cc = j - dy * sp.len;
            const int tx = cc < sp.na ? sp.ax0 + cc : sp.bx0 + (cc - sp.na);
            ++total;
            if (slr::span_index(sp, sp.ty0 + dy, tx) != j) ++bad;
        }
    }
    std::printf("checked %ld slots, %ld mismatches\n", total, bad);
    return bad != 0;
}
