// Host-only table construction of libsqueeze (declarations and the data
// layouts in host_tables.h).  No HIP: compiled by g++.
#include "host_tables.h"

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <utility>

namespace sqz {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local char g_err[512];

sqz_status set_error(sqz_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

const char *last_error_text() { return g_err; }

// ---------------------------------------------------------------------------
// Invariant division
// ---------------------------------------------------------------------------
Div32 make_div32(uint32_t d)
{
    Div32 D;
    D.d = d;
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    D.m = (uint32_t)((((unsigned __int128)1 << 32) * (((unsigned __int128)1 << l) - d)) / d + 1);
    D.sh1 = l < 1 ? l : 1;
    D.sh2 = l > 0 ? l - 1 : 0;
    return D;
}

Div64 make_div64(uint64_t d)
{
    Div64 D;
    D.d = d;
    uint32_t l = 0;
    while (l < 64 && ((unsigned __int128)1 << l) < d) ++l;
    D.m = (uint64_t)((((unsigned __int128)1 << 64) * (((unsigned __int128)1 << l) - d)) / d + 1);
    D.sh1 = l < 1 ? l : 1;
    D.sh2 = l > 0 ? l - 1 : 0;
    return D;
}

static uint64_t upow(uint64_t b, int e)
{
    uint64_t p = 1;
    while (e-- > 0) p *= b;
    return p;
}

// ---------------------------------------------------------------------------
// Descriptor
// ---------------------------------------------------------------------------
sqz_status check_descriptor(int32_t s, int32_t k, const int32_t *offs, int32_t r, FractalHost *F)
{
    if (s < 2 || s > kMaxS) return set_error(SQZ_ERR_INVALID, "s=%d outside [2, %d]", s, kMaxS);
    if (k < 1 || k > s * s) return set_error(SQZ_ERR_INVALID, "k=%d outside [1, s*s=%d]", k, s * s);
    if (!offs) return set_error(SQZ_ERR_INVALID, "offsets_xy is NULL");
    if (r < 0) return set_error(SQZ_ERR_INVALID, "r=%d is negative", r);
    int seen[kMaxS * kMaxS];
    for (int i = 0; i < s * s; ++i) seen[i] = -1;
    for (int j = 0; j < k; ++j) {
        const int x = offs[2 * j], y = offs[2 * j + 1];
        if (x < 0 || x >= s || y < 0 || y >= s)
            return set_error(SQZ_ERR_INVALID, "replica %d offset (%d,%d) outside [0,%d)^2", j, x, y, s);
        if (seen[x + s * y] >= 0)
            return set_error(SQZ_ERR_INVALID, "replicas %d and %d share offset (%d,%d)", seen[x + s * y], j, x, y);
        seen[x + s * y] = j;
    }
    // n = s^r < 2^31, N = k^r < 2^62
    uint64_t n = 1, N = 1;
    for (int i = 0; i < r; ++i) {
        n *= (uint64_t)s;
        if (n >= (1ull << 31)) return set_error(SQZ_ERR_RANGE, "n = %d^%d does not fit in 31 bits", s, r);
        N *= (uint64_t)k;
        if (N >= (1ull << 62)) return set_error(SQZ_ERR_RANGE, "N = %d^%d does not fit in 62 bits", k, r);
    }
    if (F) {
        memset(F, 0, sizeof *F);
        F->s = s;
        F->k = k;
        F->r = r;
        F->n = (int64_t)n;
        F->N = N;
        for (int j = 0; j < k; ++j) {
            F->ox[j] = offs[2 * j];
            F->oy[j] = offs[2 * j + 1];
        }
        for (int i = 0; i < s * s; ++i) F->hnu[i] = seen[i];
    }
    return SQZ_OK;
}

// ---------------------------------------------------------------------------
// Map tables
// ---------------------------------------------------------------------------
// Chunk sizes: at most 4096 entries per table, lambda offsets packed in 16
// bits per axis, nu chunk values below 2^31.
static int lam_chunk(int s, int k)
{
    int c = 1;
    while (c < 24 && upow(k, c + 1) <= 4096 && upow(s, c + 1) <= 65536) ++c;
    return c;
}
static int nu_chunk(int s, int k)
{
    int c = 1;
    while (c < 24 && upow(s, 2 * (c + 1)) <= 4096 && upow(k, c + 1) < (1ull << 31)) ++c;
    return c;
}

void map_tables(const FractalHost &F, int level, MapParams &P, MapTables &T)
{
    const int s = F.s, k = F.k;
    memset(&P, 0, sizeof P);
    P.s = s;
    P.k = k;
    P.r = level;
    P.n = (int32_t)upow(s, level);
    P.N = upow(k, level);
    const int CL = lam_chunk(s, k), CN = nu_chunk(s, k);
    P.nlam = level == 0 ? 0 : (level + CL - 1) / CL;
    P.nnu = level == 0 ? 0 : (level + CN - 1) / CN;
    const int TL = level == 0 ? 0 : level - CL * (P.nlam - 1);
    const int TN = level == 0 ? 0 : level - CN * (P.nnu - 1);
    P.klam = (uint32_t)upow(k, CL);
    P.slam = (uint32_t)upow(s, CL);
    P.snu = (uint32_t)upow(s, CN);
    P.snu_top = (uint32_t)upow(s, TN);
    P.knu = upow(k, CN);
    P.dklam64 = make_div64(P.klam);
    P.dklam32 = make_div32(P.klam);
    P.dsnu = make_div32(P.snu);

    // lambda tables: digit chunk -> packed (x | y << 16)
    auto lam_table = [&](int levels, std::vector<uint32_t> &t) {
        const uint64_t cnt = upow(k, levels);
        t.resize(cnt);
        for (uint64_t d = 0; d < cnt; ++d) {
            uint64_t v = d, sp = 1, x = 0, y = 0;
            for (int i = 0; i < levels; ++i) {
                const int beta = (int)(v % k);
                v /= k;
                x += F.ox[beta] * sp;
                y += F.oy[beta] * sp;
                sp *= s;
            }
            t[d] = (uint32_t)(x | (y << 16));
        }
    };
    // nu tables: (xc + side*yc) -> base-k replica digits, or hole
    auto nu_table = [&](int levels, std::vector<uint32_t> &t) {
        const uint64_t side = upow(s, levels);
        t.resize(side * side);
        for (uint64_t yc = 0; yc < side; ++yc)
            for (uint64_t xc = 0; xc < side; ++xc) {
                uint64_t v = 0, kp = 1, sx = xc, sy = yc;
                bool hole = false;
                for (int i = 0; i < levels; ++i) {
                    const int j = F.hnu[(sx % s) + s * (sy % s)];
                    sx /= s;
                    sy /= s;
                    if (j < 0) {
                        hole = true;
                        break;
                    }
                    v += (uint64_t)j * kp;
                    kp *= k;
                }
                t[xc + side * yc] = hole ? kNuHole32 : (uint32_t)v;
            }
    };
    std::vector<uint32_t> parts[4];
    if (level > 0) {
        lam_table(CL, parts[0]);
        lam_table(TL, parts[1]);
        nu_table(CN, parts[2]);
        nu_table(TN, parts[3]);
    } else {
        for (auto &p : parts) p.assign(1, 0);
    }
    T.all.clear();
    for (int i = 0; i < 4; ++i) {
        T.off[i] = T.all.size();
        T.all.insert(T.all.end(), parts[i].begin(), parts[i].end());
    }
    P.ntab = (uint32_t)T.all.size();
}

void host_lambda(const FractalHost &F, int level, uint64_t c, int64_t &x, int64_t &y)
{
    int64_t px = 0, py = 0, sp = 1;
    for (int mu = 1; mu <= level; ++mu) {
        const int b = (int)(c % (uint64_t)F.k);
        c /= (uint64_t)F.k;
        px += F.ox[b] * sp;
        py += F.oy[b] * sp;
        sp *= F.s;
    }
    x = px;
    y = py;
}

int64_t host_nu(const FractalHost &F, int level, int64_t x, int64_t y)
{
    int64_t side = 1;
    for (int i = 0; i < level; ++i) side *= F.s;
    if (x < 0 || y < 0 || x >= side || y >= side) return -1;
    int64_t c = 0, kp = 1;
    for (int mu = 1; mu <= level; ++mu) {
        const int j = F.hnu[(int)(x % F.s) + F.s * (int)(y % F.s)];
        if (j < 0) return -1;
        c += j * kp;
        kp *= F.k;
        x /= F.s;
        y /= F.s;
    }
    return c;
}

static int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Bit-sliced tiles
// ---------------------------------------------------------------------------
sqz_status tile_tables(const FractalHost &F, const TileSpec &S, TileTables &T)
{
    const int M = S.M, J = S.J;
    const uint64_t tile = upow(F.k, M), nblocks = upow(F.k, M - J);
    const int64_t side = (int64_t)upow(F.s, M), box = S.box;

    // ring 1: cells of adjacent tiles that touch a cell of this tile
    struct Slot {
        int dx, dy;
        int64_t idx, px, py;  // cell index in the neighbour tile; position relative to this tile
    };
    std::vector<Slot> ring;
    auto find = [&](int64_t qx, int64_t qy) {
        for (size_t i = 0; i < ring.size(); ++i)
            if (ring[i].px == qx && ring[i].py == qy) return (int64_t)i;
        return (int64_t)-1;
    };
    auto outside_member = [&](int64_t qx, int64_t qy, int &tdx, int &tdy) {
        tdx = qx < 0 ? -1 : (qx >= side ? 1 : 0);
        tdy = qy < 0 ? -1 : (qy >= side ? 1 : 0);
        return host_nu(F, M, qx - tdx * side, qy - tdy * side);
    };
    for (uint64_t c = 0; c < tile; ++c) {
        int64_t x, y;
        host_lambda(F, M, c, x, y);
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int64_t qx = x + dx, qy = y + dy;
                if (qx >= 0 && qy >= 0 && qx < side && qy < side) continue;
                int tdx, tdy;
                const int64_t j = outside_member(qx, qy, tdx, tdy);
                if (j >= 0 && find(qx, qy) < 0) ring.push_back(Slot{tdx, tdy, j, qx, qy});
            }
    }
    if (ring.size() > (size_t)S.max_tile_halo)
        return set_error(SQZ_ERR_UNSUPPORTED, "tile halo of %zu cells exceeds %d", ring.size(), S.max_tile_halo);
    T.nthalo = (uint32_t)ring.size();

    // rings 2..max_steps (several steps per launch): breadth-first from ring 1
    // over member cells outside the tile (ring d = graph distance d from the
    // tile); all rings must fit max_ring lanes, and ring cells must lie in the
    // adjacent tiles (d < side).
    std::vector<uint32_t> start = {0, (uint32_t)ring.size()};
    uint32_t ksteps = 1;
    for (int d = 2; d <= S.max_steps; ++d) {
        for (uint32_t c = start[d - 2]; c < start[d - 1]; ++c)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int64_t qx = ring[c].px + dx, qy = ring[c].py + dy;
                    if (qx >= 0 && qy >= 0 && qx < side && qy < side) continue;
                    int tdx, tdy;
                    const int64_t j = outside_member(qx, qy, tdx, tdy);
                    if (j >= 0 && find(qx, qy) < 0) ring.push_back(Slot{tdx, tdy, j, qx, qy});
                }
        start.push_back((uint32_t)ring.size());
        if (T.nthalo == 0 || start[d] > (uint32_t)S.max_ring || d >= side) break;
        ksteps = (uint32_t)d;  // rings 1..d fit: d steps per launch
    }
    T.ksteps = ksteps;
    for (int d = 0; d <= S.max_steps && d < 16; ++d) T.ring_start[d] = start[d <= (int)ksteps ? d : ksteps];
    T.tstride = T.ring_start[ksteps];
    T.nsrc = ksteps >= 2 ? T.ring_start[ksteps - 1] : 0;
    ring.resize(T.tstride);

    // adjacent blocks of other tiles that hold ring-1 cells (one LDS word each)
    std::vector<std::pair<int64_t, int64_t>> vblk;
    auto virt_of = [&](int64_t bx, int64_t by) {
        for (size_t g = 0; g < vblk.size(); ++g)
            if (vblk[g].first == bx && vblk[g].second == by) return (int64_t)g;
        return (int64_t)-1;
    };
    for (uint32_t i = 0; i < T.nthalo; ++i) {
        const int64_t bx = floor_div(ring[i].px, box), by = floor_div(ring[i].py, box);
        if (virt_of(bx, by) < 0) vblk.emplace_back(bx, by);
    }
    // LDS entry (byte offset of the word << 16 | bit) of a tile cell and of ring cell i
    auto entry = [](uint32_t word, uint32_t bit) { return (4u * word) << 16 | bit; };
    const uint32_t zero_entry = entry(S.lds_zero, 0);
    auto tile_entry = [&](int64_t j) { return entry((uint32_t)(j / S.nc), (uint32_t)(j % S.nc)); };
    auto ring_entry = [&](size_t i) {
        uint32_t d = 1;
        while ((uint32_t)i >= T.ring_start[d]) ++d;
        if (d == 1) {
            const Slot &s = ring[i];
            const int64_t g = virt_of(floor_div(s.px, box), floor_div(s.py, box));
            return entry(S.lds_virt + (uint32_t)g, (uint32_t)(s.idx % S.nc));
        }
        const uint32_t k = (uint32_t)i - T.nthalo;  // rings 2.. packed in order
        return entry(S.lds_ring2 + k / 32, k % 32);
    };
    T.home.assign(T.tstride ? T.tstride : 1, zero_entry);
    for (uint32_t i = 0; i < T.tstride; ++i) T.home[i] = ring_entry(i);
    // LDS sources of the neighbours of every ring cell that is advanced
    T.rsrc.assign(T.nsrc ? (size_t)T.nsrc * 8 : 1, zero_entry);
    for (uint32_t c = 0; c < T.nsrc; ++c) {
        int n = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy) continue;
                const int64_t qx = ring[c].px + dx, qy = ring[c].py + dy;
                uint32_t e = zero_entry;
                if (qx >= 0 && qy >= 0 && qx < side && qy < side) {
                    const int64_t j = host_nu(F, M, qx, qy);
                    if (j >= 0) e = tile_entry(j);
                } else {
                    int tdx, tdy;
                    if (outside_member(qx, qy, tdx, tdy) >= 0) {
                        const int64_t i = find(qx, qy);  // always a loaded ring cell: ring d-1, d or d+1
                        if (i >= 0 && i < (int64_t)T.tstride) e = ring_entry((size_t)i);
                    }
                }
                T.rsrc[(size_t)c * 8 + n++] = e;
            }
    }

    // adjacent-block words of every block: a block of the tile, the word of
    // an adjacent block of another tile, or a zero word (no such block)
    const int NG = S.ngrp, NP = (NG + 1) / 2;
    T.nbstride = NP > 4 ? (uint32_t)((NP + 3) / 4 * 4) : 4u;
    T.nbt.assign((size_t)nblocks * T.nbstride, 0);
    const int64_t bside = (int64_t)upow(F.s, M - J);
    for (uint64_t b = 0; b < nblocks; ++b) {
        int64_t bx, by;
        host_lambda(F, M - J, b, bx, by);
        for (int g = 0; g < NG; ++g) {
            const int64_t nbx = bx + S.g_dx[g], nby = by + S.g_dy[g];
            uint32_t w = S.lds_zero;
            if (nbx >= 0 && nby >= 0 && nbx < bside && nby < bside) {
                const int64_t nb = host_nu(F, M - J, nbx, nby);
                if (nb >= 0) w = (uint32_t)nb;
            } else {
                const int64_t v = virt_of(nbx, nby);
                if (v >= 0) w = S.lds_virt + (uint32_t)v;
            }
            T.nbt[(size_t)b * T.nbstride + g / 2] |= (4u * w) << (16 * (g & 1));
        }
    }

    // per ring cell: adjacent-tile offset and the cell's index in that tile
    T.slots.assign(T.tstride ? (size_t)T.tstride * 4 : 4, 0);
    for (uint32_t i = 0; i < T.tstride; ++i) {
        T.slots[4 * i] = ring[i].dx;
        T.slots[4 * i + 1] = ring[i].dy;
        T.slots[4 * i + 2] = (int32_t)ring[i].idx;
    }
    // the tile's own cells that any tile loads as ring cells: every index that
    // appears in a ring slot (the slot tables are the same for every tile)
    std::vector<uint8_t> used(tile, 0);
    for (uint32_t i = 0; i < T.tstride; ++i) used[(size_t)ring[i].idx] = 1;
    T.bound.clear();
    for (uint64_t j = 0; j < tile; ++j)
        if (used[j]) T.bound.push_back((uint32_t)j);
    return SQZ_OK;
}

// ---------------------------------------------------------------------------
// Expanded tiles
// ---------------------------------------------------------------------------
void xtile_ring_slots(const FractalHost &F, int M, uint32_t P, std::vector<XRingSlot> &out)
{
    const int64_t side = (int64_t)upow(F.s, M);
    const uint64_t KM = upow(F.k, M);
    std::vector<uint8_t> seen((size_t)P * P, 0);
    out.clear();
    for (uint64_t c = 0; c < KM; ++c) {
        int64_t x, y;
        host_lambda(F, M, c, x, y);
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int64_t qx = x + dx, qy = y + dy;
                if (qx >= 0 && qy >= 0 && qx < side && qy < side) continue;
                const int tdx = qx < 0 ? -1 : (qx >= side ? 1 : 0), tdy = qy < 0 ? -1 : (qy >= side ? 1 : 0);
                const int64_t j = host_nu(F, M, qx - tdx * side, qy - tdy * side);
                if (j < 0) continue;
                const uint32_t pos = (uint32_t)((qy + 1) * P + (qx + 1));
                if (seen[pos]) continue;
                seen[pos] = 1;
                const int d = (tdy + 1) * 3 + (tdx + 1);
                const uint32_t d8 = (uint32_t)(d < 4 ? d : d - 1);
                out.push_back(XRingSlot{(uint16_t)pos, (d8 << 16) | (uint32_t)j});
            }
    }
}

void xtile_cell_entries(const FractalHost &F, int M, uint32_t P, const int field_shift[8],
                        std::vector<uint16_t> &lam, std::vector<uint32_t> &ent)
{
    const int64_t side = (int64_t)upow(F.s, M);
    const uint64_t KM = upow(F.k, M);
    lam.assign(KM, 0);
    ent.assign(KM, 0);
    for (uint64_t c = 0; c < KM; ++c) {
        int64_t x, y;
        host_lambda(F, M, c, x, y);
        lam[c] = (uint16_t)((y + 1) * P + (x + 1));
        // member neighbours inside the tile, and per adjacent tile the member
        // cells of that tile (its own copy of the level-M pattern) it touches
        uint32_t inner = 0, cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0) continue;
                const int64_t qx = x + dx, qy = y + dy;
                const int tdx = qx < 0 ? -1 : (qx >= side ? 1 : 0), tdy = qy < 0 ? -1 : (qy >= side ? 1 : 0);
                const bool member = host_nu(F, M, qx - tdx * side, qy - tdy * side) >= 0;
                if (!member) continue;
                if (tdx == 0 && tdy == 0) {
                    ++inner;
                } else {
                    const int d = (tdy + 1) * 3 + (tdx + 1);
                    ++cnt[d < 4 ? d : d - 1];
                }
            }
        uint32_t e = lam[c] | inner << 16;
        for (int d8 = 0; d8 < 8; ++d8) e |= cnt[d8] << field_shift[d8];  // sides <= 3, corners <= 1
        ent[c] = e;
    }
}

void xtile_layer_tables(const FractalHost &F, int M, int K, uint32_t P, uint32_t rows,
                        std::vector<XRingSlot> &ring, std::vector<uint32_t> &start, std::vector<uint16_t> &lam,
                        std::vector<uint8_t> &mem)
{
    const int64_t B = (int64_t)upow(F.s, M);
    const uint64_t KM = upow(F.k, M);
    ring.clear();
    start.assign(1, 0);
    // ring slots by layer: member cells of the adjacent tiles within K of the box
    for (int d = 1; d <= K; ++d) {
        for (int64_t qy = -K; qy < B + K; ++qy)
            for (int64_t qx = -K; qx < B + K; ++qx) {
                const int64_t ex = qx < 0 ? -qx : (qx >= B ? qx - B + 1 : 0);
                const int64_t ey = qy < 0 ? -qy : (qy >= B ? qy - B + 1 : 0);
                if ((ex > ey ? ex : ey) != d) continue;
                const int tdx = qx < 0 ? -1 : (qx >= B ? 1 : 0), tdy = qy < 0 ? -1 : (qy >= B ? 1 : 0);
                const int64_t j = host_nu(F, M, qx - tdx * B, qy - tdy * B);
                if (j < 0) continue;
                const int dd = (tdy + 1) * 3 + (tdx + 1);
                const uint32_t d8 = (uint32_t)(dd < 4 ? dd : dd - 1);
                ring.push_back(XRingSlot{(uint16_t)((qy + K) * P + (qx + K)), (d8 << 16) | (uint32_t)j});
            }
        start.push_back((uint32_t)ring.size());
    }
    // box positions of the tile's cells and their membership
    lam.assign(KM, 0);
    mem.assign((size_t)P * rows, 0);
    for (uint64_t c = 0; c < KM; ++c) {
        int64_t x, y;
        host_lambda(F, M, c, x, y);
        lam[c] = (uint16_t)((y + K) * P + (x + K));
        mem[lam[c]] = 1;
    }
}

// ---------------------------------------------------------------------------
// Bit-row tiles
// ---------------------------------------------------------------------------
void bitbox_tables(const FractalHost &F, const BitboxSpec &S, std::vector<uint16_t> &bpos,
                   std::vector<uint32_t> &ring, std::vector<uint32_t> &member)
{
    const int M = S.M, BD = S.border;
    const uint64_t nblk = upow(F.k, M - 1);
    const int64_t sb = (int64_t)upow(3, M - 1), GB = sb + 2 * BD;

    // grid positions of the tile's blocks
    bpos.assign(nblk, 0);
    for (uint64_t b = 0; b < nblk; ++b) {
        int64_t x, y;
        host_lambda(F, M - 1, b, x, y);
        bpos[b] = (uint16_t)((x + BD) | (y + BD) << 7);
    }
    // border blocks: position in an adjacent tile, if a block of the pattern is there
    auto outside_block = [&](int64_t gx, int64_t gy, int &dir) -> int64_t {
        const int64_t bx = gx - BD, by = gy - BD;
        const int64_t tdx = floor_div(bx, sb), tdy = floor_div(by, sb);
        dir = (int)((tdy + 1) * 3 + (tdx + 1));
        return host_nu(F, M - 1, bx - tdx * sb, by - tdy * sb);
    };
    ring.clear();
    for (int64_t gy = 0; gy < GB; ++gy)
        for (int64_t gx = 0; gx < GB; ++gx) {
            const bool inner = gx >= BD && gy >= BD && gx < BD + sb && gy < BD + sb;
            if (inner) continue;
            int dir;
            const int64_t lb = outside_block(gx, gy, dir);
            if (lb >= 0) ring.push_back((uint32_t)(gy * S.grid_pitch + gx) | (uint32_t)dir << 14 | (uint32_t)lb << 18);
        }
    // membership of every box position (adjacent tiles present)
    member.assign((size_t)S.rows * S.words, 0);
    for (int64_t cy = 0; cy < 3 * GB; ++cy)
        for (int64_t cx = 0; cx < 3 * GB; ++cx) {
            if (F.hnu[(int)(cx % 3) + 3 * (int)(cy % 3)] < 0) continue;
            const int64_t gx = cx / 3, gy = cy / 3;
            const bool inner = gx >= BD && gy >= BD && gx < BD + sb && gy < BD + sb;
            int dir;
            const int64_t lb = inner ? host_nu(F, M - 1, gx - BD, gy - BD) : outside_block(gx, gy, dir);
            if (lb >= 0) member[(size_t)cy * S.words + cx / 32] |= 1u << (cx % 32);
        }
}

}  // namespace sqz
