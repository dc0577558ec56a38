// Host-side check of the block -> (tile, right-hand-side group) maps of the
// hop and fused normal kernels (hop.hpp): for every map, run of time slices,
// block size and group count on a set of lattice shapes, the grid that
// tile_map_blocks sizes covers every (tile, group) pair exactly once, and
// time_run keeps its stated window.  Built and run on the CPU by
// test_tile_map_host.py; it launches nothing on a GPU.
#include <cstdio>
#include <vector>

#include "hop.hpp"

using namespace lqs;

int main()
{
    const int dims[][4] = {{4, 4, 4, 4},    {4, 6, 8, 10},   {2, 4, 2, 6},     {8, 8, 8, 16},    {16, 16, 16, 16},
                           {24, 24, 24, 8}, {24, 24, 24, 24}, {32, 32, 32, 8}, {32, 32, 32, 32}, {32, 16, 4, 8},
                           {32, 32, 4, 6},  {48, 48, 48, 12}, {64, 64, 64, 16}};
    long cases = 0, bad = 0;
    for (const auto &d : dims) {
        Geom g;
        for (int i = 0; i < 4; ++i) g.n[i] = d[i];
        g.vh = d[0] * d[1] * d[2] * d[3] / 2;
        for (int block : {64, 128, 256, 512})
            for (int mode : {-1, 0, 1, 2, 3})
                for (int run : {0, 1, 2, 3, 4, 8, 100})
                    for (int G : {1, 2, 3, 4}) {
                        const TileMap m = tile_map(g, block, mode, run);
                        const unsigned nb = tile_map_blocks(g, block, m, G);
                        const int tiles = (g.vh + block - 1) / block;
                        std::vector<int> seen((size_t)tiles * G, 0);
                        bool ok = true;
                        for (unsigned b = 0; b < nb; ++b) {
                            int grp = -1;
                            const int t = tile_of_block((int)b, G, m, g.n[3], grp);
                            if (t < 0 || (long)t * block >= g.vh) continue;  // padding block
                            if (grp < 0 || grp >= G) {
                                ok = false;
                                continue;
                            }
                            seen[(size_t)t * G + grp] += 1;
                        }
                        for (int c : seen) ok = ok && c == 1;
                        ++cases;
                        if (!ok) {
                            ++bad;
                            std::printf("BAD dims %dx%dx%dx%d block %d mode %d run %d G %d kind %d\n", d[0], d[1], d[2],
                                        d[3], block, mode, run, G, m.kind);
                        }
                    }
        // time_run: explicit runs pass through; all slices up to Nt = 8; else a run of 2..8
        // whose z-reuse window (2 run tiles, all sides) is within 2 MiB unless already 2
        for (int nrhs : {1, 4, 16})
            for (int prec : {F64, F32, F16}) {
                const int r = time_run(g, 256, nrhs, prec, -1);
                const long win = 2l * r * 256 * nrhs * spinor_bytes_per_site(prec);
                const bool ok = (g.n[3] <= 8) ? r == 0 : (r >= 2 && r <= 8 && (win <= (2l << 20) || r == 2));
                ++cases;
                if (!ok || time_run(g, 256, nrhs, prec, 3) != 3) {
                    ++bad;
                    std::printf("BAD time_run dims %dx%dx%dx%d nrhs %d prec %d -> %d\n", d[0], d[1], d[2], d[3], nrhs,
                                prec, r);
                }
            }
    }
    std::printf("cases %ld bad %ld\n", cases, bad);
    return bad ? 1 : 0;
}
