// CPU check of the compile-time block plans of the bit-sliced tiled kernels
// (tile_device.h): for random block words and adjacent-block words, the
// bit-sliced layers the plan builds must give every cell of the block exactly
// its number of live Moore neighbours (counted by brute force from the
// cells' positions), with no two contributions to one cell in one layer.
// Host code only; no GPU call.
#include <cstdio>
#include <random>

#include "tile_device.h"

using namespace sqz;

template <class Pat>
static int check(const char *name)
{
    constexpr const BlockPlan &P = PlanOf<Pat>::value;
    std::mt19937 rng(2201);
    int bad = 0;
    const uint32_t cells = P.nc == 32 ? 0xFFFFFFFFu : ((1u << P.nc) - 1u);
    for (int it = 0; it < 20000; ++it) {
        const uint32_t x = rng() & cells;
        uint32_t w[8];
        for (int g = 0; g < 8; ++g) w[g] = rng();
        uint32_t L[8] = {};
        for (int t = 0; t < P.nterm; ++t) {
            const uint32_t v = (P.t_shift[t] > 0 ? x >> P.t_shift[t] : x << -P.t_shift[t]) & P.t_mask[t];
            bad += (L[P.t_layer[t]] & P.t_mask[t]) != 0;  // a layer bit set twice
            L[P.t_layer[t]] |= v;
        }
        for (int t = 0; t < P.nhterm; ++t) {
            const int g = P.h_grp[P.ht_slot[t]], src = P.h_idx[P.ht_slot[t]], bit = P.ht_bit[t];
            bad += (L[P.ht_layer[t]] >> bit) & 1u & ((w[g] >> src) & 1u);
            L[P.ht_layer[t]] |= ((w[g] >> src) & 1u) << bit;
        }
        for (int i = 0; i < P.nc; ++i) {
            int got = 0, want = 0;
            for (int l = 0; l < P.nlayer; ++l) got += (L[l] >> i) & 1;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy) continue;
                    const int qx = P.lx[i] + dx, qy = P.ly[i] + dy;
                    if (qx >= 0 && qy >= 0 && qx < P.box && qy < P.box) {
                        const int j = local_nu<Pat>(qx, qy);
                        if (j >= 0) want += (x >> j) & 1;
                    } else {
                        const int bdx = qx < 0 ? -1 : (qx >= P.box ? 1 : 0), bdy = qy < 0 ? -1 : (qy >= P.box ? 1 : 0);
                        const int j = local_nu<Pat>(qx - bdx * P.box, qy - bdy * P.box);
                        if (j < 0) continue;
                        int g = -1;
                        for (int q = 0; q < P.ngrp; ++q)
                            if (P.g_dx[q] == bdx && P.g_dy[q] == bdy) g = q;
                        want += g < 0 ? 1000 : (int)((w[g] >> j) & 1u);
                    }
                }
            bad += got != want;
        }
    }
    printf("%s: %d cells per block, %d in-block moves, %d halo moves, %d layers, %d mismatches\n", name, P.nc, P.nterm,
           P.nhterm, P.nlayer, bad);
    return bad;
}

int main()
{
    const int bad = check<PatTriangle>("triangle") + check<PatTriangleBig>("triangle (level-10 tiles)") +
                    check<PatTrianglePaper>("triangle, paper orientation") + check<PatVicsek>("Vicsek cross");
    if (!bad) printf("all checks passed\n");
    return bad ? 1 : 0;
}
