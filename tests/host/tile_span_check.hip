// Host-side check of the tile placement of the tiled step (tile_span in
// goc_tile.hpp): for every axis length n in [3, 700), tile size T of the
// built shapes and either boundary kind, the tiles of the axis together own
// every node exactly once, each tile's extent lies in the axis and covers
// the nodes it owns, and next to a wall the three nodes of a one-sided
// difference lie in the tile.  Prints "ok" or the first failure.
#include <cstdio>

#include "goc_tile.hpp"

int main()
{
    const int sizes[] = {4, 8, 16, 64, 128};
    for (int T : sizes)
        for (int n = 3; n < 700; ++n)
            for (int periodic = 0; periodic < 2; ++periodic) {
                const int tiles = (n + T - 1) / T;
                int owned_total = 0;
                for (int b = 0; b < tiles; ++b) {
                    const int o = b * T, hi = o + T < n ? o + T : n;   // owned nodes [o, hi)
                    int ext = 0, org = 0;
                    goc::tile_span(n, T, o, periodic != 0, ext, org);
                    const bool ok_span = ext >= 1 && ext <= T && org >= 0 && org + ext <= n;
                    const bool ok_cover = org <= o && org + ext >= hi;
                    const bool ok_far = periodic || hi < n || n - 3 >= org;   // one-sided at n - 1
                    const bool ok_near = periodic || o > 0 || org + ext >= 3;  // one-sided at 0
                    if (!(ok_span && ok_cover && ok_far && ok_near)) {
                        std::printf("fail T=%d n=%d periodic=%d tile=%d ext=%d org=%d\n", T, n, periodic, b, ext, org);
                        return 1;
                    }
                    owned_total += hi - o;
                }
                if (owned_total != n) {
                    std::printf("fail T=%d n=%d periodic=%d: %d nodes owned\n", T, n, periodic, owned_total);
                    return 1;
                }
            }
    std::printf("ok\n");
    return 0;
}
