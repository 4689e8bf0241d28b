// CPU checks of libsqueeze's host-only table builders (host_tables.cpp),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py.  Every table is compared with brute force
// over the pattern: a mismatch prints a message and exits non-zero; a
// sanitizer report aborts.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <set>
#include <utility>
#include <vector>

#include "host_tables.h"

using namespace sqz;

static int g_fail = 0;
#define EXPECT(cond, ...)                                   \
    do {                                                    \
        if (!(cond)) {                                      \
            fprintf(stderr, "FAILED %s:%d: ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);                   \
            fprintf(stderr, "\n");                          \
            if (++g_fail > 20) exit(1);                     \
        }                                                   \
    } while (0)

struct Pattern {
    const char *name;
    int s, k;
    int offs[16];
};
static const Pattern kPatterns[] = {
    {"triangle", 2, 3, {0, 0, 1, 0, 0, 1}},
    {"triangle_paper", 2, 3, {0, 0, 0, 1, 1, 1}},
    {"carpet", 3, 8, {0, 0, 1, 0, 2, 0, 0, 1, 2, 1, 0, 2, 1, 2, 2, 2}},
    {"vicsek", 3, 5, {1, 0, 0, 1, 1, 1, 2, 1, 1, 2}},
};

static int64_t ipow(int64_t b, int e)
{
    int64_t p = 1;
    while (e-- > 0) p *= b;
    return p;
}

static FractalHost make(const Pattern &p, int r)
{
    FractalHost F;
    const sqz_status st = check_descriptor(p.s, p.k, p.offs, r, &F);
    EXPECT(st == SQZ_OK, "%s r=%d: %s", p.name, r, last_error_text());
    return F;
}

// Membership and compact index by replication (level 0: the origin; level mu:
// k copies of level mu-1 at offset tau_j s^(mu-1)).
static std::vector<std::pair<int64_t, int64_t>> replicate(const FractalHost &F, int level)
{
    std::vector<std::pair<int64_t, int64_t>> v(1, {0, 0});
    int64_t sc = 1;
    for (int mu = 1; mu <= level; ++mu) {
        std::vector<std::pair<int64_t, int64_t>> w;
        for (int j = 0; j < F.k; ++j)
            for (auto &c : v) w.push_back({c.first + F.ox[j] * sc, c.second + F.oy[j] * sc});
        v.swap(w);
        sc *= F.s;
    }
    return v;
}

static void check_divisions()
{
    const uint32_t ds[] = {1, 2, 3, 5, 7, 8, 9, 25, 27, 81, 125, 243, 729, 2187, 4096, 6561, 59049, 531441, 0x7FFFFFFFu,
                           0xFFFFFFFFu};
    uint64_t x = 88172645463325252ull;
    for (uint32_t d : ds) {
        const Div32 D = make_div32(d);
        const Div64 E = make_div64(d);
        for (int i = 0; i < 20000; ++i) {
            x ^= x << 13;
            x ^= x >> 7;
            x ^= x << 17;
            const uint32_t n = i < 8 ? (uint32_t)(0xFFFFFFFFu - i) : (i < 16 ? (uint32_t)(i - 8) : (uint32_t)x);
            const uint32_t t = (uint32_t)(((uint64_t)D.m * n) >> 32);
            const uint32_t q = (t + ((n - t) >> D.sh1)) >> D.sh2;
            EXPECT(q == n / d, "div32 %u / %u: %u", n, d, q);
            const uint64_t n64 = i < 8 ? ~0ull - (uint64_t)i : x;
            const uint64_t t64 = (uint64_t)(((unsigned __int128)E.m * n64) >> 64);
            const uint64_t q64 = (t64 + ((n64 - t64) >> E.sh1)) >> E.sh2;
            EXPECT(q64 == n64 / d, "div64 %llu / %u", (unsigned long long)n64, d);
        }
    }
}

static void check_descriptors()
{
    FractalHost F;
    const int bad_offs[] = {0, 0, 0, 0};
    EXPECT(check_descriptor(2, 2, bad_offs, 3, &F) == SQZ_ERR_INVALID, "duplicate offsets accepted");
    EXPECT(check_descriptor(1, 1, bad_offs, 3, &F) == SQZ_ERR_INVALID, "s=1 accepted");
    EXPECT(check_descriptor(17, 1, bad_offs, 3, &F) == SQZ_ERR_INVALID, "s=17 accepted");
    EXPECT(check_descriptor(2, 5, bad_offs, 3, &F) == SQZ_ERR_INVALID, "k > s^2 accepted");
    EXPECT(check_descriptor(2, 1, nullptr, 3, &F) == SQZ_ERR_INVALID, "NULL offsets accepted");
    EXPECT(check_descriptor(2, 1, bad_offs, -1, &F) == SQZ_ERR_INVALID, "r < 0 accepted");
    const int out_offs[] = {0, 2};
    EXPECT(check_descriptor(2, 1, out_offs, 3, &F) == SQZ_ERR_INVALID, "offset outside [0,s) accepted");
    EXPECT(check_descriptor(2, 3, kPatterns[0].offs, 31, &F) == SQZ_ERR_RANGE, "n = 2^31 accepted");
    EXPECT(check_descriptor(2, 3, kPatterns[0].offs, 30, &F) == SQZ_OK, "n = 2^30 refused");
    EXPECT(check_descriptor(16, 256, nullptr, 1, &F) == SQZ_ERR_INVALID, "NULL offsets accepted (k=256)");
    std::vector<int> all(512);
    for (int i = 0; i < 256; ++i) {
        all[2 * i] = i % 16;
        all[2 * i + 1] = i / 16;
    }
    EXPECT(check_descriptor(16, 256, all.data(), 7, &F) == SQZ_OK, "full 16x16 pattern refused");
    EXPECT(check_descriptor(16, 256, all.data(), 8, &F) == SQZ_ERR_RANGE, "256^8 accepted");
    EXPECT(check_descriptor(3, 8, kPatterns[2].offs, 19, &F) == SQZ_OK && F.N == (uint64_t)ipow(8, 19), "carpet r=19");
}

// lambda and nu through the chunk tables, evaluated the way the kernels do.
static void check_maps(const Pattern &p, int r)
{
    const FractalHost F = make(p, r);
    MapParams P;
    MapTables T;
    map_tables(F, r, P, T);
    const uint32_t *lam_lo = T.all.data() + T.off[0], *lam_top = T.all.data() + T.off[1];
    const uint32_t *nu_lo = T.all.data() + T.off[2], *nu_top = T.all.data() + T.off[3];
    const size_t n_lam_lo = T.off[1] - T.off[0], n_lam_top = T.off[2] - T.off[1];
    const size_t n_nu_lo = T.off[3] - T.off[2], n_nu_top = T.all.size() - T.off[3];
    EXPECT(P.N == (uint64_t)ipow(p.k, r) && P.n == ipow(p.s, r), "%s r=%d sizes", p.name, r);
    const auto cells = replicate(F, r);
    std::vector<int64_t> dense((size_t)(P.n + 2) * (P.n + 2), -1);
    for (size_t c = 0; c < cells.size(); ++c) {
        // lambda through the tables
        uint64_t v = c;
        uint32_t px = 0, py = 0, sp = 1;
        for (int i = 0; i + 1 < P.nlam; ++i) {
            const uint64_t q = v / P.klam;
            const size_t e = (size_t)(v - q * P.klam);
            EXPECT(e < n_lam_lo, "lam_lo index");
            px += (lam_lo[e] & 0xFFFFu) * sp;
            py += (lam_lo[e] >> 16) * sp;
            v = q;
            sp *= P.slam;
        }
        if (P.nlam > 0) {
            EXPECT(v < n_lam_top, "%s r=%d lam_top index %llu", p.name, r, (unsigned long long)v);
            if (v < n_lam_top) {
                px += (lam_top[v] & 0xFFFFu) * sp;
                py += (lam_top[v] >> 16) * sp;
            }
        }
        EXPECT(px == cells[c].first && py == cells[c].second, "%s r=%d lambda(%zu)", p.name, r, c);
        int64_t hx, hy;
        host_lambda(F, r, c, hx, hy);
        EXPECT(hx == cells[c].first && hy == cells[c].second, "%s r=%d host_lambda(%zu)", p.name, r, c);
        dense[(size_t)(cells[c].second + 1) * (P.n + 2) + (cells[c].first + 1)] = (int64_t)c;
    }
    // nu over the box and a one-cell ring around it
    for (int64_t y = -1; y <= P.n; ++y)
        for (int64_t x = -1; x <= P.n; ++x) {
            const int64_t want = dense[(size_t)(y + 1) * (P.n + 2) + (x + 1)];
            int64_t got = -1;
            if (x >= 0 && y >= 0 && x < P.n && y < P.n) {
                uint32_t ux = (uint32_t)x, uy = (uint32_t)y;
                uint64_t c = 0, kp = 1;
                bool hole = false;
                for (int i = 0; i + 1 < P.nnu && !hole; ++i) {
                    const uint32_t qx = ux / P.snu, qy = uy / P.snu;
                    const size_t idx = (ux - qx * P.snu) + (size_t)P.snu * (uy - qy * P.snu);
                    EXPECT(idx < n_nu_lo, "nu_lo index");
                    const uint32_t e = nu_lo[idx];
                    if (e == kNuHole32) hole = true;
                    c += (uint64_t)e * kp;
                    kp *= P.knu;
                    ux = qx;
                    uy = qy;
                }
                if (!hole && P.nnu > 0) {
                    const size_t idx = ux + (size_t)P.snu_top * uy;
                    EXPECT(idx < n_nu_top, "nu_top index");
                    const uint32_t e = nu_top[idx];
                    if (e == kNuHole32) hole = true;
                    c += (uint64_t)e * kp;
                }
                got = hole ? -1 : (int64_t)c;
                if (P.nnu == 0) got = 0;
            }
            EXPECT(got == want, "%s r=%d nu(%lld,%lld) = %lld, want %lld", p.name, r, (long long)x, (long long)y,
                   (long long)got, (long long)want);
            EXPECT(host_nu(F, r, x, y) == want, "%s r=%d host_nu(%lld,%lld)", p.name, r, (long long)x, (long long)y);
        }
}

// Bit-sliced tile tables of the triangle (blocks of level 3, all eight
// adjacent-block directions): ring sizes, slot positions, LDS entries.
static void check_tiles(int M, const uint32_t *want_rings, int nwant)
{
    const FractalHost F = make(kPatterns[0], M + 3);
    TileSpec S;
    memset(&S, 0, sizeof S);
    S.M = M;
    S.J = 3;
    S.nc = 27;
    S.box = 8;
    S.ngrp = 8;
    int g = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx)
            if (dx || dy) {
                S.g_dx[g] = dx;
                S.g_dy[g] = dy;
                ++g;
            }
    const uint32_t nblocks = (uint32_t)ipow(3, M - 3);
    S.lds_zero = nblocks;
    S.lds_virt = nblocks + 2;
    S.lds_ring2 = nblocks + 2 + 32;
    S.max_tile_halo = 32;
    S.max_ring = 256;
    S.max_steps = 10;
    TileTables T;
    EXPECT(tile_tables(F, S, T) == SQZ_OK, "tile_tables M=%d: %s", M, last_error_text());
    EXPECT(T.ksteps == 10, "M=%d ksteps %u", M, T.ksteps);
    for (int d = 1; d <= nwant; ++d)
        EXPECT(T.ring_start[d] - T.ring_start[d - 1] == want_rings[d - 1], "M=%d ring %d: %u cells, want %u", M, d,
               T.ring_start[d] - T.ring_start[d - 1], want_rings[d - 1]);
    const int64_t side = ipow(2, M);
    // every ring slot is a member of an adjacent tile at graph distance d from the tile
    std::set<std::pair<int64_t, int64_t>> seen;
    for (uint32_t i = 0; i < T.tstride; ++i) {
        const int dx = T.slots[4 * i], dy = T.slots[4 * i + 1], idx = T.slots[4 * i + 2];
        EXPECT((dx || dy) && dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1, "slot %u direction", i);
        EXPECT(idx >= 0 && idx < ipow(3, M), "slot %u index", i);
        int64_t x, y;
        host_lambda(F, M, (uint64_t)idx, x, y);
        x += dx * side;
        y += dy * side;
        EXPECT(seen.insert({x, y}).second, "slot %u repeated", i);
        // ring 1 cells touch the tile
        if (i < T.nthalo) {
            bool touch = false;
            for (int ey = -1; ey <= 1; ++ey)
                for (int ex = -1; ex <= 1; ++ex)
                    touch |= host_nu(F, M, x + ex, y + ey) >= 0;
            EXPECT(touch, "ring-1 slot %u does not touch the tile", i);
        }
        EXPECT((T.home[i] >> 16) % 4 == 0 && (T.home[i] & 0xFFFF) < 32, "home entry %u", i);
    }
    // LDS entries of advanced ring cells stay inside the tile's words
    const uint32_t words = S.lds_ring2 + (256 + 31) / 32;
    for (uint32_t i = 0; i < T.nsrc * 8; ++i) EXPECT((T.rsrc[i] >> 16) / 4 < words, "rsrc entry %u", i);
    for (uint32_t b = 0; b < nblocks; ++b)
        for (int q = 0; q < S.ngrp; ++q) {
            const uint32_t w = (T.nbt[(size_t)b * T.nbstride + q / 2] >> (16 * (q & 1))) & 0xFFFFu;
            EXPECT(w % 4 == 0 && w / 4 < S.lds_ring2, "nbt block %u group %d: %u", b, q, w);
        }
    // boundary list: every index a slot names, once, in order
    std::set<uint32_t> idx;
    for (uint32_t i = 0; i < T.tstride; ++i) idx.insert((uint32_t)T.slots[4 * i + 2]);
    EXPECT(idx.size() == T.bound.size() && std::equal(idx.begin(), idx.end(), T.bound.begin()), "bound list M=%d", M);
}

static void check_xtiles(const Pattern &p, int M)
{
    const FractalHost F = make(p, M + 2);
    const int64_t B = ipow(p.s, M);
    const uint32_t P = (uint32_t)((B + 2 + 3) / 4 * 4);
    std::vector<XRingSlot> ring;
    xtile_ring_slots(F, M, P, ring);
    std::set<uint16_t> pos;
    for (const XRingSlot &r : ring) {
        EXPECT(pos.insert(r.pos).second, "%s M=%d repeated ring position", p.name, M);
        const int64_t qx = (int64_t)(r.pos % P) - 1, qy = (int64_t)(r.pos / P) - 1;
        EXPECT(qx < 0 || qy < 0 || qx >= B || qy >= B, "%s ring slot inside the tile", p.name);
        EXPECT((r.info >> 16) < 8 && (r.info & 0xFFFF) < ipow(p.k, M), "%s ring info", p.name);
    }
    int shifts[8] = {20, 22, 24, 26, 28, 29, 30, 31};
    std::vector<uint16_t> lam;
    std::vector<uint32_t> ent;
    xtile_cell_entries(F, M, P, shifts, lam, ent);
    for (size_t c = 0; c < lam.size(); ++c) {
        EXPECT((ent[c] & 0xFFFF) == lam[c], "%s entry position", p.name);
        int64_t x, y;
        host_lambda(F, M, c, x, y);
        int inner = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                if ((dx || dy) && host_nu(F, M, x + dx, y + dy) >= 0) ++inner;
        EXPECT((int)((ent[c] >> 16) & 15) == inner, "%s cell %zu inner count", p.name, c);
    }
    for (int K = 2; K <= 3; ++K) {
        const uint32_t PK = (uint32_t)((B + 2 * K + 3) / 4 * 4), rows = (uint32_t)(B + 2 * K);
        std::vector<XRingSlot> lr;
        std::vector<uint32_t> start;
        std::vector<uint16_t> lamk;
        std::vector<uint8_t> mem;
        xtile_layer_tables(F, M, K, PK, rows, lr, start, lamk, mem);
        EXPECT((int)start.size() == K + 1 && start.back() == lr.size(), "%s layer starts", p.name);
        size_t members = 0;
        for (uint8_t m : mem) members += m;
        EXPECT(members == (size_t)ipow(p.k, M), "%s membership count", p.name);
    }
}

static void check_bitbox(int M)
{
    const FractalHost F = make(kPatterns[2], M + 2);
    BitboxSpec S;
    S.M = M;
    S.border = 4;
    S.grid_pitch = 100;
    S.rows = 270;
    S.words = 9;
    std::vector<uint16_t> bpos;
    std::vector<uint32_t> ring, member;
    bitbox_tables(F, S, bpos, ring, member);
    EXPECT(bpos.size() == (size_t)ipow(8, M - 1), "bitbox blocks");
    std::set<uint16_t> pos(bpos.begin(), bpos.end());
    EXPECT(pos.size() == bpos.size(), "bitbox repeated block position");
    const int64_t sb = ipow(3, M - 1), GB = sb + 8;
    for (uint32_t r : ring) {
        const uint32_t g = r & 0x3FFF, dir = (r >> 14) & 15, lb = r >> 18;
        EXPECT(g % 100 < GB && g / 100 < GB && dir < 9 && dir != 4 && lb < ipow(8, M - 1), "bitbox ring entry");
    }
    size_t bits = 0;
    for (uint32_t w : member) bits += (size_t)__builtin_popcount(w);
    // members in the box: the tile's cells plus those of the adjacent tiles inside the border
    size_t want = 0;
    for (int64_t cy = 0; cy < 3 * GB; ++cy)
        for (int64_t cx = 0; cx < 3 * GB; ++cx) {
            const int64_t x = cx - 12, y = cy - 12, side = 3 * sb;
            const int64_t tx = x < 0 ? -1 : (x >= side ? 1 : 0), ty = y < 0 ? -1 : (y >= side ? 1 : 0);
            want += host_nu(F, M, x - tx * side, y - ty * side) >= 0;
        }
    EXPECT(bits == want, "bitbox membership %zu, want %zu", bits, want);
}

int main()
{
    check_divisions();
    check_descriptors();
    for (const Pattern &p : kPatterns)
        for (int r = 0; r <= (p.s == 2 ? 9 : 5); ++r) check_maps(p, r);
    const uint32_t rings8[10] = {8, 14, 14, 22, 18, 28, 24, 38, 18, 28};
    check_tiles(8, rings8, 10);
    check_tiles(10, rings8, 10);
    for (const Pattern &p : kPatterns)
        for (int M = 1; M <= (p.s == 2 ? 7 : 4); ++M) check_xtiles(p, M);
    for (int M = 3; M <= 5; ++M) check_bitbox(M);
    if (g_fail) {
        fprintf(stderr, "%d check(s) failed\n", g_fail);
        return 1;
    }
    printf("host tables: all checks passed\n");
    return 0;
}
