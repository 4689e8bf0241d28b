// Block-level Squeeze (Section "Moving from Thread-level to Block-level")
// for Life on compact storage, bit-sliced.
//
// Work decomposition
//   tile  = a level-M subtree: the contiguous compact range [t K^M, (t+1) K^M).
//           One workgroup per tile.  The coarse maps (lambda/nu at level r-M)
//           are evaluated once per tile, ahead of time, to find the few cells of
//           neighbouring tiles that touch it ("tile halo").
//   block = a level-J subtree of K^J <= 32 cells, held as one 32-bit word
//           (bit i = state of the block's cell i).  One lane per block.
// Inside a tile nothing is mapped per cell: the neighbours of a block's cells
// are either cells of the same block -- a fixed set of (bit shift, bit mask)
// moves derived from the replica pattern at compile time -- or fixed cells
// ("block halo") of a few adjacent blocks, whose words are found through a
// table that is the same for every tile (the micro brute force the paper
// applies inside a block).  Neighbour counts are summed with bit-sliced full
// adders over up to eight single-bit layers, then B3/S23 is applied to all
// cells of the block with a few logic operations.
//
// Memory path per tile: coalesced 16-byte loads of the tile's bytes, packed to
// bits in LDS (pack: a 4-byte dot product with byte weights 1,2,4,8 (then
// 16..128) turns eight 0/1 bytes into one byte of bits), cut into one word
// per block; results are joined back into 32-cell words and written with
// coalesced 16-byte stores (unpack: (v * 0x204081) & 0x01010101 spreads four
// bits over four bytes).  Tile boundaries are not 16-byte aligned: the two
// edge words of a tile are stored byte by byte, one byte per lane, so
// neighbouring tiles never overwrite each other.
#pragma once

#include <type_traits>
#include <utility>

#include "common.h"

namespace sqz {

// ---------------------------------------------------------------------------
// Replica patterns with a tiled kernel.  Replica j is at (OX[j], OY[j]).
// ---------------------------------------------------------------------------
// Build-time knobs (defaults are the tuned values).
#ifndef SQZ_TRI_TILE_LEVEL  // triangle tile level for large fractals (512-lane workgroups)
#define SQZ_TRI_TILE_LEVEL 10
#endif
#ifndef SQZ_TRI_TILE_BIG_FROM  // fractal level from which triangle tiles use SQZ_TRI_TILE_LEVEL (else 8)
#define SQZ_TRI_TILE_BIG_FROM 16
#endif
#ifndef SQZ_SPLIT_EXCHANGE  // 1: the resident run updates interior blocks while its exchange barrier completes
#define SQZ_SPLIT_EXCHANGE 1
#endif
#ifndef SQZ_NT_LOAD
#define SQZ_NT_LOAD 0
#endif
#ifndef SQZ_NT_STORE  // 1: nontemporal stores in every tiled kernel, 0: in the multi-step kernels only
#define SQZ_NT_STORE 0
#endif

// Tile level M: MMAX for fractals of level >= MBIG, else MSMALL (more,
// smaller tiles keep a smaller fractal's launch balanced; from level 16 the
// larger triangle tile is faster with several steps per launch).  Large
// triangles are their own pattern type, with level-10 tiles and 512-lane
// workgroups (all of a level-16 triangle's 729 tiles resident at once), so
// that the kernels for smaller triangles (and the batch) keep LDS sized for
// level-8 tiles.
struct PatTriangle {  // Sierpinski triangle, member iff x & y == 0
    static constexpr int S = 2, K = 3, J = 3, MMAX = 8, MSMALL = 8, MBIG = 0;
    static constexpr int OX[3] = {0, 1, 0};
    static constexpr int OY[3] = {0, 0, 1};
};
struct PatTriangleBig {  // the same pattern, fractal level >= SQZ_TRI_TILE_BIG_FROM
    static constexpr int S = 2, K = 3, J = 3, MMAX = SQZ_TRI_TILE_LEVEL, MSMALL = SQZ_TRI_TILE_LEVEL, MBIG = 0;
    static constexpr int OX[3] = {0, 1, 0};
    static constexpr int OY[3] = {0, 0, 1};
};
struct PatTrianglePaper {  // the paper's orientation: top, middle, right
    static constexpr int S = 2, K = 3, J = 3, MMAX = 9, MSMALL = 8, MBIG = SQZ_TRI_TILE_BIG_FROM;
    static constexpr int OX[3] = {0, 0, 1};
    static constexpr int OY[3] = {0, 1, 1};
};
struct PatVicsek {  // Vicsek cross
    static constexpr int S = 3, K = 5, J = 2, MMAX = 6, MSMALL = 6, MBIG = 0;
    static constexpr int OX[5] = {1, 0, 1, 2, 1};
    static constexpr int OY[5] = {0, 1, 1, 1, 2};
};

constexpr int cpow(int b, int e)
{
    int p = 1;
    for (int i = 0; i < e; ++i) p *= b;
    return p;
}

constexpr int kMaxHalo = 16;      // halo cells per block
constexpr int kMaxSteps = 10;     // Life steps per launch of the multi-step tiled kernel
constexpr int kMaxTileHalo = 32;  // halo cells per tile (one LDS word of bits)
constexpr int kMaxRing = 256;     // ring cells of all rings (one lane each)
constexpr int kRingTab = kMaxRing * 9;  // LDS words of a tile's ring tables: 8 sources per cell, then homes
constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Compile-time plan of one block's neighbourhood.
// ---------------------------------------------------------------------------
struct BlockPlan {
    int nc, box;
    int lx[32], ly[32];              // local lambda of the block's cells
    int nlayer;                      // single-bit layers summed per cell
    int nterm;                       // in-block moves: L[layer] |= shift(x) & mask
    int t_layer[128], t_shift[128];  // shift > 0: source bit above target (x >> shift)
    uint32_t t_mask[128];
    int nhalo;                       // distinct halo cells (block direction, cell)
    int h_dx[kMaxHalo], h_dy[kMaxHalo], h_idx[kMaxHalo];
    int nhterm;                      // L[layer] |= halo_bit[slot] << bit
    int ht_layer[64], ht_slot[64], ht_bit[64];
    int ngrp;                        // distinct adjacent blocks holding halo cells
    int g_dx[8], g_dy[8];
    int h_grp[kMaxHalo];             // adjacent block of each halo cell
    bool ok;
};

template <class Pat>
constexpr int local_nu(int x, int y)
{
    int c = 0;
    for (int mu = Pat::J; mu >= 1; --mu) {
        const int sc = cpow(Pat::S, mu - 1);
        const int qx = (x / sc) % Pat::S, qy = (y / sc) % Pat::S;
        int j = -1;
        for (int i = 0; i < Pat::K; ++i)
            if (Pat::OX[i] == qx && Pat::OY[i] == qy) j = i;
        if (j < 0) return -1;
        c += j * cpow(Pat::K, mu - 1);
    }
    return c;
}

// Layer colouring of the in-block moves: every distinct shift (source bit
// index minus target bit index) gets one layer, such that two shifts that
// reach a common target bit get different layers (graph colouring by
// backtracking, at most 8 layers).  Then each shift is a single move term
// whose mask holds all its target bits.  Returns the number of layers, 0 if
// no colouring with at most 8 layers exists.
struct ShiftColouring {
    int nsh;
    int sh[64];
    bool conf[64][64];
    int col[64];
};

constexpr bool colour_from(ShiftColouring &c, const int (&order)[64], int idx, int k)
{
    if (idx == c.nsh) return true;
    const int a = order[idx];
    for (int col = 0; col < k; ++col) {
        bool ok = true;
        for (int b = 0; b < c.nsh && ok; ++b)
            if (c.conf[a][b] && c.col[b] == col) ok = false;
        if (!ok) continue;
        c.col[a] = col;
        if (colour_from(c, order, idx + 1, k)) return true;
        c.col[a] = -1;
    }
    return false;
}

template <class Pat>
constexpr BlockPlan derive_plan()
{
    BlockPlan p{};
    p.ok = true;
    p.nc = cpow(Pat::K, Pat::J);
    p.box = cpow(Pat::S, Pat::J);
    if (p.nc > 32) {
        p.ok = false;
        return p;
    }
    for (int i = 0; i < p.nc; ++i) {
        int v = i, x = 0, y = 0, sp = 1;
        for (int mu = 1; mu <= Pat::J; ++mu) {
            const int b = v % Pat::K;
            v /= Pat::K;
            x += Pat::OX[b] * sp;
            y += Pat::OY[b] * sp;
            sp *= Pat::S;
        }
        p.lx[i] = x;
        p.ly[i] = y;
    }
    // in-block shifts and their conflicts (two shifts reaching one target bit)
    ShiftColouring c{};
    int tshift[32][8] = {};
    int ntshift[32] = {};
    for (int i = 0; i < p.nc; ++i)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy) continue;
                const int qx = p.lx[i] + dx, qy = p.ly[i] + dy;
                if (qx < 0 || qy < 0 || qx >= p.box || qy >= p.box) continue;
                const int j = local_nu<Pat>(qx, qy);
                if (j < 0) continue;
                int a = -1;
                for (int q = 0; q < c.nsh; ++q)
                    if (c.sh[q] == j - i) a = q;
                if (a < 0) {
                    a = c.nsh++;
                    c.sh[a] = j - i;
                }
                tshift[i][ntshift[i]++] = a;
            }
    for (int i = 0; i < p.nc; ++i)
        for (int u = 0; u < ntshift[i]; ++u)
            for (int w = 0; w < ntshift[i]; ++w)
                if (u != w) c.conf[tshift[i][u]][tshift[i][w]] = true;
    int order[64] = {};
    int degc[64] = {};
    for (int a = 0; a < c.nsh; ++a) {
        order[a] = a;
        c.col[a] = -1;
        for (int b = 0; b < c.nsh; ++b) degc[a] += c.conf[a][b] ? 1 : 0;
    }
    for (int u = 1; u < c.nsh; ++u)  // most-constrained shift first
        for (int w = u; w > 0 && degc[order[w]] > degc[order[w - 1]]; --w) {
            const int t = order[w];
            order[w] = order[w - 1];
            order[w - 1] = t;
        }
    int maxdeg = 0;
    for (int i = 0; i < p.nc; ++i) maxdeg = ntshift[i] > maxdeg ? ntshift[i] : maxdeg;
    bool coloured = false;
    for (int k = maxdeg < 1 ? 1 : maxdeg; k <= 8 && !coloured; ++k) {
        for (int a = 0; a < c.nsh; ++a) c.col[a] = -1;
        coloured = colour_from(c, order, 0, k);
    }
    for (int i = 0; i < p.nc; ++i) {
        bool used[8] = {};
        int nused = 0;
        int halo_slots[8] = {};
        int nh = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy) continue;
                const int qx = p.lx[i] + dx, qy = p.ly[i] + dy;
                if (qx >= 0 && qy >= 0 && qx < p.box && qy < p.box) {
                    const int j = local_nu<Pat>(qx, qy);
                    if (j < 0) continue;
                    const int shift = j - i;  // source bit j -> target bit i
                    int layer = -1;
                    if (coloured) {  // the shift's own layer and term
                        for (int a = 0; a < c.nsh; ++a)
                            if (c.sh[a] == shift) layer = c.col[a];
                        int t = -1;
                        for (int q = 0; q < p.nterm; ++q)
                            if (p.t_shift[q] == shift) t = q;
                        if (t < 0) {
                            t = p.nterm++;
                            p.t_layer[t] = layer;
                            p.t_shift[t] = shift;
                            p.t_mask[t] = 0;
                        }
                        p.t_mask[t] |= 1u << i;
                    } else {  // greedy: a term of this shift whose layer is free for bit i
                        for (int t = 0; t < p.nterm && layer < 0; ++t)
                            if (p.t_shift[t] == shift && !used[p.t_layer[t]]) {
                                layer = p.t_layer[t];
                                p.t_mask[t] |= 1u << i;
                            }
                        if (layer < 0) {
                            for (int l = 0; l < 8 && layer < 0; ++l)
                                if (!used[l]) layer = l;
                            p.t_layer[p.nterm] = layer;
                            p.t_shift[p.nterm] = shift;
                            p.t_mask[p.nterm] = 1u << i;
                            ++p.nterm;
                        }
                    }
                    used[layer] = true;
                    ++nused;
                } else {
                    const int bdx = qx < 0 ? -1 : (qx >= p.box ? 1 : 0);
                    const int bdy = qy < 0 ? -1 : (qy >= p.box ? 1 : 0);
                    const int j = local_nu<Pat>(qx - bdx * p.box, qy - bdy * p.box);
                    if (j < 0) continue;
                    int slot = -1;
                    for (int h = 0; h < p.nhalo; ++h)
                        if (p.h_dx[h] == bdx && p.h_dy[h] == bdy && p.h_idx[h] == j) slot = h;
                    if (slot < 0) {
                        if (p.nhalo == kMaxHalo) {
                            p.ok = false;
                            return p;
                        }
                        slot = p.nhalo++;
                        p.h_dx[slot] = bdx;
                        p.h_dy[slot] = bdy;
                        p.h_idx[slot] = j;
                    }
                    halo_slots[nh++] = slot;
                }
            }
        for (int h = 0; h < nh; ++h) {
            int layer = -1;
            for (int l = 0; l < 8 && layer < 0; ++l)
                if (!used[l]) layer = l;
            if (layer < 0) {
                p.ok = false;
                return p;
            }
            used[layer] = true;
            ++nused;
            p.ht_layer[p.nhterm] = layer;
            p.ht_slot[p.nhterm] = halo_slots[h];
            p.ht_bit[p.nhterm] = i;
            ++p.nhterm;
        }
        for (int l = 0; l < 8; ++l)
            if (used[l] && l + 1 > p.nlayer) p.nlayer = l + 1;
        if (nused > p.nlayer) p.nlayer = nused;
    }
    for (int h = 0; h < p.nhalo; ++h) {
        int g = -1;
        for (int q = 0; q < p.ngrp; ++q)
            if (p.g_dx[q] == p.h_dx[h] && p.g_dy[q] == p.h_dy[h]) g = q;
        if (g < 0) {
            g = p.ngrp++;
            p.g_dx[g] = p.h_dx[h];
            p.g_dy[g] = p.h_dy[h];
        }
        p.h_grp[h] = g;
    }
    return p;
}

template <class Pat>
struct PlanOf {
    static constexpr BlockPlan value = derive_plan<Pat>();
    static_assert(value.ok, "replica pattern does not fit the bit-sliced block kernel");
};

// ---------------------------------------------------------------------------
// Per-tile configuration built on the host.
// ---------------------------------------------------------------------------
struct TileConfig {
    int M;                 // tile level
    uint32_t tile;         // K^M cells per tile
    uint32_t nblocks;      // K^(M-J)
    uint32_t nthalo;       // tile halo slots (ring 1: cells of other tiles adjacent to the tile)
    uint32_t ksteps;       // Life steps one launch of the multi-step kernel can take (1: none)
    uint32_t ring_start[kMaxSteps + 1];  // slots of ring d are [ring_start[d-1], ring_start[d])
    uint32_t nsrc;         // ring cells whose next states are computed: ring_start[ksteps - 1]
    uint32_t tstride;      // per-tile entries of d_tile_halo: ring_start[ksteps]
    uint32_t nbstride;     // u32 entries per block in d_nbtab (multiple of 4)
    uint64_t ntiles;       // K^(r-M)
    uint32_t *d_nbtab;     // [nblocks][nbstride] LDS byte offsets (16-bit pairs) of each block's adjacent-block words
    uint64_t *d_tile_halo; // [ntiles][tstride] global indices of the ring cells
    uint32_t *d_ringsrc;   // [nsrc][8] LDS sources of each advanced ring cell's neighbours
    uint32_t *d_ringhome;  // [tstride] LDS word and bit of each ring cell
    MapParams Pc;          // maps at the coarse level r-M
    void *d_coarse_tables;
    // resident run (all tiles on the chip at once), null / 0 when unavailable
    uint32_t nbound;       // boundary cells per tile (exported at every exchange)
    uint32_t lds_pad;      // LDS bytes reserved per workgroup so that at most ceil(tiles / CUs) share a CU
    uint32_t *d_bound;     // [nbound] their tile-local indices
    uint32_t *d_bar;       // {arrivals, timed out} of the grid barrier
    uint32_t *h_flag;      // pinned host word: a barrier wait of an earlier run timed out
};

struct TileArgs {
    uint64_t ntiles, N;
    uint32_t tile, nblocks, nthalo, tstride, nsrc, nbstride;
    uint32_t ring_start[kMaxSteps + 1];
    const uint32_t *nbtab;
    const uint64_t *tile_halo;
    const uint32_t *ringsrc;
    const uint32_t *ringhome;
};

inline TileArgs tile_args(const FractalHost &F)
{
    const TileConfig *T = F.tile;
    TileArgs A;
    A.ntiles = T->ntiles;
    A.N = F.N;
    A.tile = T->tile;
    A.nblocks = T->nblocks;
    A.nthalo = T->nthalo;
    A.tstride = T->tstride;
    A.nsrc = T->nsrc;
    A.nbstride = T->nbstride;
    for (int d = 0; d <= kMaxSteps; ++d) A.ring_start[d] = T->ring_start[d];
    A.nbtab = T->d_nbtab;
    A.tile_halo = T->d_tile_halo;
    A.ringsrc = T->d_ringsrc;
    A.ringhome = T->d_ringhome;
    return A;
}

// LDS words of one tile's state, one word per level-J block (bit i = cell i
// of the block, bits from K^J up zero): blocks [0, NBMAX), two words that
// stay zero (absent neighbours), one word per adjacent block of another tile
// that holds ring-1 cells (each at its bit within that block), then the bits
// of rings 2..kMaxSteps, packed in ring order.  Ring d holds the cells of other
// tiles at graph distance d from the tile (each neighbour of a ring-d cell is
// in ring d-1, d or d+1, or in the tile for d = 1).  The layout does not
// depend on where the tile starts within a 32-byte word, so every table that
// addresses it is the same for all tiles.  The tile's bytes are first packed
// to bits at their 32-byte alignment in the low words of another buffer
// (STAGE words) and then cut into block words.
template <class Pat>
struct TileLds {
    static constexpr int NC = PlanOf<Pat>::value.nc;
    static constexpr int TMAX = cpow(Pat::K, Pat::MMAX);
    static constexpr int NBMAX = TMAX / NC;
    static constexpr int ZERO = NBMAX;
    static constexpr int VIRT = ZERO + 2;
    static constexpr int RING2 = VIRT + kMaxTileHalo;
    static constexpr int WORDS = RING2 + (kMaxRing + 31) / 32;
    static constexpr int STAGE = (TMAX + 31 + 31) / 32 + 1;
    static constexpr int NGRP = PlanOf<Pat>::value.ngrp > 0 ? PlanOf<Pat>::value.ngrp : 1;
    static_assert(STAGE <= NBMAX, "packed tile overlaps the special words");
    static_assert(NC > 16, "a 32-bit word must span at most three blocks");
};

// LDS entry: byte offset of a word within a buffer << 16 | bit.
__device__ __forceinline__ uint32_t lds_bit(const uint32_t *base, uint32_t e)
{
    return __builtin_amdgcn_ubfe(*reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(base) + (e >> 16)),
                                 e, 1);
}
__device__ __forceinline__ uint32_t *lds_word(uint32_t *base, uint32_t e)
{
    return reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(base) + (e >> 16));
}

// Bit 0 of eight bytes (two words) -> one byte of bits, via 4-byte dot products.
__device__ __forceinline__ uint32_t pack8(uint32_t d0, uint32_t d1)
{
    return __builtin_amdgcn_udot4(d1, 0x80402010u, __builtin_amdgcn_udot4(d0, 0x08040201u, 0u, false), false);
}
__device__ __forceinline__ uint32_t spread4(uint32_t v) { return __umul24(v, 0x204081u) & 0x01010101u; }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 load16(const uint8_t *p)
{
#if SQZ_NT_LOAD
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
#else
    return *reinterpret_cast<const uint4 *>(p);
#endif
}
template <bool NTS>
__device__ __forceinline__ void store16(uint8_t *p, uint4 v)
{
    if constexpr (NTS || SQZ_NT_STORE) {
        u32x4 w = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(w, reinterpret_cast<u32x4 *>(p));
    } else {
        *reinterpret_cast<uint4 *>(p) = v;
    }
}

// (a << S) | c as one instruction.  Written out because the compiler
// rewrites ((a & m) << s) | c into a shift, an AND with the shifted mask and
// a separate OR (and folds a single-bit extract into the shift after it).
template <int S>
__device__ __forceinline__ uint32_t lshl_or(uint32_t a, uint32_t c)
{
    if constexpr (S == 0) {
        return a | c;
    } else {
        uint32_t d;
        asm("v_lshl_or_b32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "i"(S), "v"(c));
        return d;
    }
}
template <int B>
__device__ __forceinline__ uint32_t bit_of(uint32_t a)
{
    return (a >> B) & 1u;
}

// One move: the cells of the block word x that reach their neighbours by a
// shift of `Shift` bits, placed into layer `Layer`.  A left move masks its
// sources first, so that the shift and the OR into the layer are one
// instruction; a single-bit right move extracts its bit and does the same.
template <int Layer, int Shift, uint32_t Mask, int NL>
__device__ __forceinline__ void move_term(uint32_t x, uint32_t (&L)[NL])
{
    if constexpr (Shift < 0)
        L[Layer] = lshl_or<-Shift>(x & (Mask >> -Shift), L[Layer]);
    else if constexpr ((Mask & (Mask - 1u)) == 0u)
        L[Layer] = lshl_or<__builtin_ctz(Mask)>(bit_of<__builtin_ctz(Mask) + Shift>(x), L[Layer]);
    else
        L[Layer] |= (x >> Shift) & Mask;
}

template <class Pat, int NL, size_t... I>
__device__ __forceinline__ void apply_moves(uint32_t x, uint32_t (&L)[NL], std::index_sequence<I...>)
{
    constexpr const BlockPlan &PL = PlanOf<Pat>::value;
    (move_term<PL.t_layer[I], PL.t_shift[I], PL.t_mask[I], NL>(x, L), ...);
}

// Halo cell `Src` of an adjacent block's word -> bit `Bit` of layer `Layer`.
template <int Layer, int Grp, int Src, int Bit, int NL, int NG>
__device__ __forceinline__ void halo_term(const uint32_t (&w)[NG], uint32_t (&L)[NL])
{
    L[Layer] = lshl_or<Bit>(bit_of<Src>(w[Grp]), L[Layer]);
}

template <class Pat, int NL, int NG, size_t... I>
__device__ __forceinline__ void apply_halo(const uint32_t (&w)[NG], uint32_t (&L)[NL], std::index_sequence<I...>)
{
    constexpr const BlockPlan &PL = PlanOf<Pat>::value;
    (halo_term<PL.ht_layer[I], PL.h_grp[PL.ht_slot[I]], PL.h_idx[PL.ht_slot[I]], PL.ht_bit[I], NL, NG>(w, L), ...);
}

// B3/S23 on all cells of a block: alive' = (count == 3) | (alive & count == 2).
template <int NL>
__device__ __forceinline__ uint32_t life_rule(uint32_t x, const uint32_t (&L)[NL])
{
    if constexpr (NL <= 5) {
        uint32_t v[5] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
        for (int l = 0; l < NL; ++l) v[l] = L[l];
        const uint32_t a = v[0], b = v[1], c = v[2], d = v[3], e = v[4];
        const uint32_t s1 = a ^ b ^ c, c1 = (a & b) | (c & (a ^ b));
        const uint32_t s2 = s1 ^ d ^ e, c2 = (s1 & d) | (e & (s1 ^ d));
        // count = s2 + 2 (c1 + c2): 2 or 3 iff exactly one carry
        return (c1 ^ c2) & (s2 | x);
    } else {
        uint32_t b0 = 0, b1 = 0, b2 = 0;  // b2 sticks once the count reaches 4
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const uint32_t c0 = b0 & L[l];
            b0 ^= L[l];
            b2 |= b1 & c0;
            b1 ^= c0;
        }
        return ~b2 & b1 & (b0 | x);
    }
}

// XCD-aware order: workgroups are dealt round-robin to the 8 XCDs; give each
// XCD a contiguous run of tiles so halo reads of adjacent tiles hit its L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t G)
{
    const uint32_t q = G / 8, rem = G % 8, xcd = b % 8, pos = b / 8;
    return xcd < rem ? xcd * (q + 1) + pos : rem * (q + 1) + (xcd - rem) * q + pos;
}

// LDS byte offsets of the adjacent-block words of this lane's blocks
// (blocks threadIdx.x + s * NT), two 16-bit offsets per register; the
// table is the same for every tile, so it is read once per tile and kept in
// registers for all steps.
template <class Pat, int NT>
struct NbRegs {
    static constexpr int NSLOT = (TileLds<Pat>::NBMAX + NT - 1) / NT;  // blocks per lane
    static constexpr int NP = (TileLds<Pat>::NGRP + 1) / 2;
    static_assert(NT % 64 == 0 && TileLds<Pat>::WORDS - TileLds<Pat>::ZERO <= NT,
                  "whole waves; special words are cleared by one pass of the workgroup");
    uint32_t a[NSLOT][NP];
    __device__ __forceinline__ uint32_t at(int s, int g) const { return g & 1 ? a[s][g >> 1] >> 16 : a[s][g >> 1] & 0xFFFFu; }
    // Keeps the compiler from unpacking the offsets once for all steps,
    // which would double the registers they take.
    __device__ __forceinline__ void keep_packed()
    {
#pragma unroll
        for (int s = 0; s < NSLOT; ++s)
#pragma unroll
            for (int p = 0; p < NP; ++p) asm volatile("" : "+v"(a[s][p]));
    }
};

#ifndef SQZ_RES_STATIC  // 1: resident rounds read LDS at fixed buffer addresses through unpacked offsets
#define SQZ_RES_STATIC 1
#endif
#ifndef SQZ_RES_UNPACK  // slots whose offsets the resident rounds hold unpacked (the rest stay packed)
#define SQZ_RES_UNPACK 3
#endif
// The same offsets, those of the first SQZ_RES_UNPACK slots one per register
// (the rest packed as in NbRegs): with the state buffer at a fixed LDS
// address, a neighbour word of an unpacked slot is read with its offset
// register as the address and the buffer in the instruction's offset field,
// without the add that unpacks and rebases a packed offset.
template <class Pat, int NT>
struct NbOffs {
    static constexpr int NSLOT = NbRegs<Pat, NT>::NSLOT;
    static constexpr int NU = SQZ_RES_UNPACK < NSLOT ? SQZ_RES_UNPACK : NSLOT;  // slots held unpacked
    static constexpr int NP = NbRegs<Pat, NT>::NP;
    uint32_t o[NU > 0 ? NU : 1][TileLds<Pat>::NGRP];
    uint32_t p[NSLOT - NU > 0 ? NSLOT - NU : 1][NP];
    __device__ __forceinline__ uint32_t at(int s, int g) const
    {
        if (s < NU) return o[s][g];
        return g & 1 ? p[s - NU][g >> 1] >> 16 : p[s - NU][g >> 1] & 0xFFFFu;
    }
    __device__ __forceinline__ void keep_packed()
    {
#pragma unroll
        for (int s = 0; s < NU; ++s)
#pragma unroll
            for (int g = 0; g < TileLds<Pat>::NGRP; ++g) asm volatile("" : "+v"(o[s][g]));
#pragma unroll
        for (int s = 0; s < NSLOT - NU; ++s)
#pragma unroll
            for (int q = 0; q < NP; ++q) asm volatile("" : "+v"(p[s][q]));
    }
};

template <class Pat, int NT>
__device__ __forceinline__ void load_nb(const TileArgs &A, NbRegs<Pat, NT> &R)
{
    constexpr int NP = NbRegs<Pat, NT>::NP;
#pragma unroll
    for (int s = 0; s < NbRegs<Pat, NT>::NSLOT; ++s) {
        const uint32_t b = threadIdx.x + s * NT;
        const uint32_t *e = A.nbtab + (size_t)(b < A.nblocks ? b : 0u) * A.nbstride;
#pragma unroll
        for (int g0 = 0; g0 < NP; g0 += 4) {
            const uint4 q = *reinterpret_cast<const uint4 *>(e + g0);
            const uint32_t qq[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int g = g0; g < NP && g < g0 + 4; ++g) R.a[s][g] = qq[g - g0];
        }
    }
}

// Phase C: one lane per level-J block.  Reads the block's word and the words
// of its adjacent blocks from `src`, writes the block's new word to `dst`.
// Full: the tile has all TileLds<Pat>::NBMAX blocks (its level is the pattern's
// largest), so every slot but the last is whole and runs without a branch,
// which lets the compiler overlap one slot's LDS reads with another's logic.
// sel (not Full): bit s set = update the blocks of slot s (the same for every
// lane of a wave).
template <class Pat, int NT, bool Full = false, class Regs = NbRegs<Pat, NT>>
__device__ __forceinline__ void tile_blocks(const TileArgs &A, Regs &R, const uint32_t *src, uint32_t *dst,
                                            uint32_t sel = ~0u)
{
    R.keep_packed();
    using LDS = TileLds<Pat>;
    constexpr const BlockPlan &PL = PlanOf<Pat>::value;
    constexpr int NC = PL.nc;
    constexpr uint32_t CELLS = NC == 32 ? 0xFFFFFFFFu : ((1u << NC) - 1u);
    constexpr int NL = PL.nlayer;
    constexpr int NG = LDS::NGRP;
    constexpr int NS = NbRegs<Pat, NT>::NSLOT;
    auto update = [&](uint32_t x, const uint32_t(&w)[NG]) {
        uint32_t L[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) L[l] = 0;
        apply_moves<Pat, NL>(x, L, std::make_index_sequence<PL.nterm>{});
        apply_halo<Pat, NL, NG>(w, L, std::make_index_sequence<PL.nhterm>{});
        return life_rule<NL>(x, L) & CELLS;
    };
    if constexpr (Full) {
        // software pipeline: the words of slot s + 1 are read before slot s is
        // updated and stored (lanes past the last block read block 0's words)
        uint32_t xc, wc[NG];
        {
            const uint32_t b = (NT <= LDS::NBMAX || threadIdx.x < A.nblocks) ? threadIdx.x : 0u;
            xc = src[b];
#pragma unroll
            for (int g = 0; g < NG; ++g)
                wc[g] = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(src) + R.at(0, g));
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const uint32_t b = threadIdx.x + s * NT;
            const uint32_t x = xc;
            uint32_t w[NG];
#pragma unroll
            for (int g = 0; g < NG; ++g) w[g] = wc[g];
            if (s + 1 < NS) {
                const uint32_t bn = threadIdx.x + (s + 1) * NT;
                xc = src[((s + 2) * NT <= LDS::NBMAX || bn < A.nblocks) ? bn : 0u];
#pragma unroll
                for (int g = 0; g < NG; ++g)
                    wc[g] = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(src) +
                                                                R.at(s + 1 < NS ? s + 1 : s, g));
            }
            const uint32_t v = update(x, w);
            if ((s + 1) * NT <= LDS::NBMAX || b < A.nblocks) dst[b] = v;
        }
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const uint32_t b = threadIdx.x + s * NT;
            if (((sel >> s) & 1u) && b < A.nblocks) {  // sel: the slots to update (uniform per wave)
                const uint32_t x = src[b];
                uint32_t w[NG];
#pragma unroll
                for (int g = 0; g < NG; ++g)
                    w[g] = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(src) + R.at(s, g));
                dst[b] = update(x, w);
            }
        }
    }
}

// Phase A: load and pack the tile (plus the bytes of its first and last
// 32-byte words that belong to the neighbouring tiles) into stg: bit i of
// word w = byte A0 + 32 w + i.
template <int NT>
__device__ __forceinline__ void tile_pack(const TileArgs &A, const uint8_t *__restrict__ in, uint64_t A0, uint32_t W,
                                          uint32_t *stg)
{
    for (uint32_t w = threadIdx.x; w < W; w += NT) {
        const uint64_t g = A0 + 32ull * w;
        uint32_t bits = 0;
        if (g + 32 <= A.N) {
            const uint4 a = load16(in + g);
            const uint4 b = load16(in + g + 16);
            bits = pack8(a.x, a.y) | pack8(a.z, a.w) << 8 | pack8(b.x, b.y) << 16 | pack8(b.z, b.w) << 24;
        } else {
            for (uint32_t i = 0; i < 32; ++i)
                if (g + i < A.N) bits |= (uint32_t)(in[g + i] & 1u) << i;
        }
        stg[w] = bits;
    }
}

// Phase A, second half: cut the packed bits (the tile starts at bit o of
// word 0) into block words.  Word W of stg (never written) only feeds bits
// that the mask drops.
template <class Pat, int NT>
__device__ __forceinline__ void tile_convert(const TileArgs &A, uint32_t o, const uint32_t *stg, uint32_t *blk)
{
    constexpr int NC = PlanOf<Pat>::value.nc;
    constexpr uint32_t CELLS = NC == 32 ? 0xFFFFFFFFu : ((1u << NC) - 1u);
    for (uint32_t b = threadIdx.x; b < A.nblocks; b += NT) {
        const uint32_t pos = o + b * NC;
        blk[b] = __builtin_amdgcn_alignbit(stg[(pos >> 5) + 1], stg[pos >> 5], pos) & CELLS;
    }
}

// Phase D: join block words back into 32-cell words, unpack and store whole
// 32-byte words (NTS: nontemporal); the (at most two) edge words of the tile
// go out byte by byte, one byte per lane of wave 0.  A whole word reads at most the blocks
// b0 .. b0+2 <= nblocks + 1; bits of blocks past the tile fall beyond bit 31.
template <class Pat, int NT, bool NTS = false>
__device__ __forceinline__ void tile_store(const TileArgs &A, uint8_t *__restrict__ out, uint64_t A0, uint32_t o,
                                           uint32_t W, const uint32_t *blk)
{
    constexpr uint32_t NC = PlanOf<Pat>::value.nc;
    const uint32_t tid = threadIdx.x, last = W - 1;
    const bool first_partial = o != 0, last_partial = ((o + A.tile) & 31) != 0;
    for (uint32_t w = tid; w < W; w += NT) {
        if (!((w == 0 && first_partial) || (w == last && last_partial))) {
            const uint32_t p0 = 32 * w - o;  // w > 0 or o == 0 here
            const uint32_t b0 = p0 / NC, r0 = p0 - b0 * NC;
            uint32_t v = (blk[b0] >> r0) | (blk[b0 + 1] << (NC - r0));
            if (2 * NC - r0 < 32) v |= blk[b0 + 2] << (2 * NC - r0);
            const uint64_t g = A0 + 32ull * w;
            uint4 a, b;
            a.x = spread4(v & 15);
            a.y = spread4((v >> 4) & 15);
            a.z = spread4((v >> 8) & 15);
            a.w = spread4((v >> 12) & 15);
            b.x = spread4((v >> 16) & 15);
            b.y = spread4((v >> 20) & 15);
            b.z = spread4((v >> 24) & 15);
            b.w = spread4(v >> 28);
            store16<NTS>(out + g, a);
            store16<NTS>(out + g + 16, b);
        }
    }
    if (tid < 64) {
        const uint32_t w = tid < 32 ? 0u : last, i = tid & 31u, lp = 32 * w + i;
        const bool mine = tid < 32 ? first_partial : (last_partial && (last != 0 || !first_partial));
        if (mine && lp >= o && lp < o + A.tile) {
            const uint32_t q = lp - o;
            out[A0 + lp] = (uint8_t)((blk[q / NC] >> (q % NC)) & 1u);
        }
    }
}

// One tile, one step.  s_in / s_out: TileLds<Pat>::WORDS words of LDS each
// (s_out first holds the packed bytes).  Called by every lane of the workgroup.
template <class Pat, int NT = kBlock>
__device__ __forceinline__ void tile_body(const TileArgs &A, const uint8_t *__restrict__ in, uint8_t *__restrict__ out,
                                          uint64_t t, uint32_t *s_in, uint32_t *s_out)
{
    using LDS = TileLds<Pat>;
    const uint32_t tid = threadIdx.x;
    const uint64_t S0 = t * A.tile;  // first byte of the tile
    const uint64_t A0 = S0 & ~31ull;
    const uint32_t o = (uint32_t)(S0 - A0);
    const uint32_t W = (o + A.tile + 31) / 32;

    // Phase B, first half: the global indices of the ring-1 cells are
    // requested before the tile's own bytes so the two latencies overlap.
    uint64_t gi = kHole64;
    uint32_t home = 0;
    if (tid < A.nthalo) {
        gi = A.tile_halo[t * A.tstride + tid];
        home = A.ringhome[tid];
    }
    NbRegs<Pat, NT> R;
    load_nb<Pat, NT>(A, R);
    tile_pack<NT>(A, in, A0, W, s_out);
    if (tid < LDS::WORDS - LDS::ZERO) s_in[LDS::ZERO + tid] = 0;
    // Phase B, second half: the ring-1 cells themselves
    uint32_t v = 0;
    if (tid < 64) v = gi != kHole64 ? (in[gi] & 1u) : 0u;
    __syncthreads();
    tile_convert<Pat, NT>(A, o, s_out, s_in);
    if (v) atomicOr(lds_word(s_in, home), 1u << (home & 31));
    __syncthreads();
    tile_blocks<Pat, NT>(A, R, s_in, s_out);
    __syncthreads();
    tile_store<Pat, NT>(A, out, A0, o, W, s_out);
    __syncthreads();  // LDS is reused by the next tile
}

// One tile, K steps (temporal blocking).  The states of the ring cells are
// loaded with the tile, one lane per ring cell; in round j (computing t+j)
// the tile's blocks and the cells of rings 1..K-j are advanced together, ring
// cell c by lane c, which reads its eight neighbours at t+j-1 (tile bits or
// ring bits, through the tile-invariant source table, copied to LDS with the
// tile).  A ring cell whose tile does not exist stays zero.  Three LDS
// buffers rotate: round j reads buf[(j-1)%3], writes buf[j%3] and clears the
// ring words of buf[(j+1)%3]; buf[2] first holds the packed bytes.  s_ring:
// kRingTab words, 16-byte aligned.
template <class Pat, int K, int NT = kBlock, bool Full = false>
__device__ __forceinline__ void tile_bodyK(const TileArgs &A, const uint8_t *__restrict__ in,
                                           uint8_t *__restrict__ out, uint64_t t, uint32_t *const buf[3],
                                           uint32_t *s_ring)
{
    using LDS = TileLds<Pat>;
    static_assert(kMaxRing <= NT, "one lane per ring cell");
    const uint32_t tid = threadIdx.x;
    const uint64_t S0 = t * A.tile;
    const uint64_t A0 = S0 & ~31ull;
    const uint32_t o = (uint32_t)(S0 - A0);
    const uint32_t W = (o + A.tile + 31) / 32;

    uint64_t gi = kHole64;
    uint32_t home = 0;
    if (tid < A.tstride) {
        gi = A.tile_halo[t * A.tstride + tid];
        home = A.ringhome[tid];
    }
    NbRegs<Pat, NT> R;
    load_nb<Pat, NT>(A, R);
    for (uint32_t i = tid; i < A.nsrc * 8; i += NT) s_ring[i] = A.ringsrc[i];
    tile_pack<NT>(A, in, A0, W, buf[2]);
    if (tid < LDS::WORDS - LDS::ZERO) {
        buf[0][LDS::ZERO + tid] = 0;
        buf[1][LDS::ZERO + tid] = 0;
        buf[2][LDS::ZERO + tid] = 0;
    }
    const bool here = gi != kHole64;  // ring cell tid exists
    uint32_t v = 0;
    if (tid < kMaxRing) {
        v = here ? (in[gi] & 1u) : 0u;
        s_ring[kMaxRing * 8 + tid] = home;
    }
    __syncthreads();
    tile_convert<Pat, NT>(A, o, buf[2], buf[0]);
    if (v) atomicOr(lds_word(buf[0], home), 1u << (home & 31));
    __syncthreads();
#pragma unroll
    for (int j = 1; j <= K; ++j) {
        const uint32_t *src = buf[(j - 1) % 3];
        uint32_t *dst = buf[j % 3];
        tile_blocks<Pat, NT, Full>(A, R, src, dst);
        if (j < K) {
            uint32_t *clr = buf[(j + 1) % 3];
            if (tid < LDS::WORDS - LDS::VIRT) clr[LDS::VIRT + tid] = 0;
            if (tid < A.ring_start[K - j]) {
                const uint4 e0 = *reinterpret_cast<const uint4 *>(s_ring + tid * 8);
                const uint4 e1 = *reinterpret_cast<const uint4 *>(s_ring + tid * 8 + 4);
                const uint32_t cnt = lds_bit(src, e0.x) + lds_bit(src, e0.y) + lds_bit(src, e0.z) +
                                     lds_bit(src, e0.w) + lds_bit(src, e1.x) + lds_bit(src, e1.y) +
                                     lds_bit(src, e1.z) + lds_bit(src, e1.w);
                const uint32_t h = s_ring[kMaxRing * 8 + tid];
                const uint32_t self = lds_bit(src, h);
                if (here & ((cnt == 3) | (self & (cnt == 2)))) atomicOr(lds_word(dst, h), 1u << (h & 31));
            }
        }
        __syncthreads();
    }
    tile_store<Pat, NT, true>(A, out, A0, o, W, buf[K % 3]);  // streaming: read next by another launch
    __syncthreads();
}


// ---------------------------------------------------------------------------
// Resident run: the tiles stay in LDS for the whole run.
//
// When every tile of the fractal fits on the chip at once (one workgroup per
// tile, all co-resident), the tile's state is loaded
// from HBM once, advanced for all steps in LDS, and stored once.  Every
// kstep steps the workgroups exchange only the cells other tiles hold as
// ring cells: each tile writes the current states of its boundary cells
// (`bound`, tile-local indices; the same for every tile) to their compact
// positions in one of the two caller buffers, the grid meets at a barrier,
// and each tile reads its ring cells from there, then advances kstep more
// steps exactly as the multi-step launch does (tile_bodyK).  Exchange
// buffers alternate between b and a, so a tile writing the exports of one
// exchange never meets a tile still reading the previous one; the final
// state goes to a (steps even) or b (odd), after one more barrier only when
// the last exchange went through that buffer.
// ---------------------------------------------------------------------------
struct ResidentArgs {
    uint8_t *a, *b;        // caller buffers; a holds the start
    int32_t steps;         // Life steps of the run (>= 1)
    int32_t kstep;         // steps between exchanges (2 .. ring depth)
    uint32_t nbound;       // boundary cells per tile
    const uint32_t *bound; // their tile-local indices
    uint32_t *bar;         // device words of the grid barrier (bar_words(grid)); counts carry over between runs
    uint32_t *flag;        // host-visible word: set to 1 when a barrier wait timed out
};

// Polls of a barrier wait before it gives up (each poll is a device-scope load
// and a short sleep, about a microsecond: seconds in all, far above any
// legitimate wait of a co-resident grid).
constexpr uint32_t kSpinLimit = 1u << 22;

// Grid barrier of a launch whose workgroups are all on the chip at once.  The
// cells the tiles exchange are written and read only with device-scope atomic
// byte accesses (stores and loads that the eight XCDs' separate L2 caches pass
// through to device-coherent memory), so no cache write-back or invalidation
// is needed: each wave waits until its exchange stores have completed, the
// workgroup meets, and one lane counts the arrival.  Counting is two-level, so
// that no counter takes more than kBarGroup atomic additions per barrier: the
// workgroups of a group of kBarGroup consecutive block indices add to their
// group's counter (own 128-byte line), the last of a group to arrive adds to
// the global counter, and every workgroup polls the global counter until all
// groups have arrived.  Counts accumulate over runs, modulo 2^32 (barrier i
// since the counters were cleared waits for i arrivals per member, compared
// wrap-safe); word 2 holds the barriers completed by earlier runs, read by
// every workgroup at its start and advanced by workgroup 0 after the run's
// last barrier, so that no run has to clear the counters (clearing them
// costs a launch of its own) and replays of a captured run stay in step.
// The workgroup meets again before any lane reads what others wrote.  The wait is bounded: after kSpinLimit polls, or as soon
// as another workgroup has given up, the workgroup marks the run as timed out
// (device word and host-visible flag) and goes on, so every wave reaches the
// end of the kernel; such a run's results are invalid and the host reports it.
constexpr uint32_t kBarGroup = 27;
constexpr uint32_t kBarStride = 32;  // words between counters (128 bytes)

__host__ __device__ constexpr uint32_t bar_words(uint64_t grid)
{
    return (uint32_t)((1 + (grid + kBarGroup - 1) / kBarGroup) * kBarStride);
}

// Arrival of this workgroup at barrier n (one lane, after the workgroup has
// met with every wave's exchange stores complete).
__device__ __forceinline__ void barrier_arrive(uint32_t *bar, uint32_t n)
{
    const uint32_t G = gridDim.x, g = blockIdx.x / kBarGroup;
    const uint32_t gs = G - g * kBarGroup < kBarGroup ? G - g * kBarGroup : kBarGroup;
    const uint32_t old = __hip_atomic_fetch_add(bar + kBarStride * (1 + g), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == n * gs) __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait of one lane until every workgroup has arrived at barrier n (bounded).
__device__ __forceinline__ void barrier_poll(uint32_t *bar, uint32_t n, uint32_t *flag)
{
    const uint32_t ng = (gridDim.x + kBarGroup - 1) / kBarGroup, target = n * ng;
    for (uint32_t spin = 0;; ++spin) {
        const uint64_t v = __hip_atomic_load(reinterpret_cast<uint64_t *>(bar), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((int32_t)((uint32_t)v - target) >= 0) break;
        if ((v >> 32) != 0 || spin == kSpinLimit) {
            __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

__device__ __forceinline__ void grid_barrier(uint32_t *bar, uint32_t nbar, uint32_t *flag)
{
    __builtin_amdgcn_s_waitcnt(0);  // this wave's exchange stores are complete
    __syncthreads();
    if (threadIdx.x == 0) {
        barrier_arrive(bar, nbar);
        barrier_poll(bar, nbar, flag);
    }
    __syncthreads();
}

// One tile for the whole run.  s_buf: three LDS buffers of TileLds<Pat>::WORDS
// words, one after another; s_ring: kRingTab words (16-byte aligned); s_rs:
// kMaxSteps + 1 words.  grid = number of tiles, all resident.
template <class Pat, int NT>
__device__ __forceinline__ void tile_bodyR(const TileArgs &A, const ResidentArgs &P, uint64_t t, uint32_t *s_buf,
                                           uint32_t *s_ring, uint32_t *s_rs)
{
    using LDS = TileLds<Pat>;
    constexpr uint32_t NC = PlanOf<Pat>::value.nc;
    constexpr uint32_t WORDS = LDS::WORDS;
    static_assert(kMaxRing <= NT, "one lane per ring cell");
    const uint32_t tid = threadIdx.x;
    const uint64_t S0 = t * A.tile;
    const uint64_t A0 = S0 & ~31ull;
    const uint32_t o = (uint32_t)(S0 - A0);
    const uint32_t W = (o + A.tile + 31) / 32;

    uint64_t gi = kHole64;
    uint32_t home = 0;
    if (tid < A.tstride) {
        gi = A.tile_halo[t * A.tstride + tid];
        home = A.ringhome[tid];
    }
    NbRegs<Pat, NT> R;
    load_nb<Pat, NT>(A, R);
    for (uint32_t i = tid; i < A.nsrc * 8; i += NT) s_ring[i] = A.ringsrc[i];
    if (tid <= (uint32_t)kMaxSteps) s_rs[tid] = A.ring_start[tid];
    tile_pack<NT>(A, P.a, A0, W, s_buf + 2 * WORDS);
    if (tid < WORDS - LDS::ZERO) {
        s_buf[LDS::ZERO + tid] = 0;
        s_buf[WORDS + LDS::ZERO + tid] = 0;
        s_buf[2 * WORDS + LDS::ZERO + tid] = 0;
    }
    const bool here = gi != kHole64;  // ring cell tid exists
    uint32_t v = 0;
    if (tid < kMaxRing) {
        v = here ? (P.a[gi] & 1u) : 0u;
        s_ring[kMaxRing * 8 + tid] = home;
    }
    __syncthreads();
    tile_convert<Pat, NT>(A, o, s_buf + 2 * WORDS, s_buf);
    if (v) atomicOr(lds_word(s_buf, home), 1u << (home & 31));
    __syncthreads();

    uint32_t cur = 0, nbar = 0;  // buffer holding the state; barriers passed in this run
    // barriers completed by earlier runs (used by the counting lane only)
    const uint32_t base = tid == 0 ? __hip_atomic_load(P.bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
    // Slots of this wave with a block that reads ring words (word VIRT and up,
    // cleared at an exchange and then filled from the other tiles): the first
    // round after an exchange updates the other slots while the barrier
    // completes, these after the ring cells have arrived.  The neighbour table
    // is the same for every tile, so this is too.
    uint32_t defer = 0;
#pragma unroll
    for (int sl = 0; sl < NbRegs<Pat, NT>::NSLOT; ++sl) {
        bool ring = false;
        if (tid + sl * NT < A.nblocks)
#pragma unroll
            for (int g = 0; g < LDS::NGRP; ++g) ring |= R.at(sl, g) >= 4u * LDS::VIRT;
        if (__ballot(ring)) defer |= 1u << sl;
    }
    // 512-lane workgroups (six waves per SIMD) have the registers for offsets held
    // unpacked; the 256-lane ones (eight) keep the packed form
    constexpr bool STATIC = SQZ_RES_STATIC && NT >= 512;
    NbOffs<Pat, NT> U;
    if constexpr (STATIC) {
#pragma unroll
        for (int sl = 0; sl < NbOffs<Pat, NT>::NU; ++sl)
#pragma unroll
            for (int g = 0; g < LDS::NGRP; ++g) U.o[sl][g] = R.at(sl, g);
#pragma unroll
        for (int sl = NbOffs<Pat, NT>::NU; sl < NbOffs<Pat, NT>::NSLOT; ++sl)
#pragma unroll
            for (int q = 0; q < NbOffs<Pat, NT>::NP; ++q) U.p[sl - NbOffs<Pat, NT>::NU][q] = R.a[sl][q];
    }
    const uint8_t *imp = nullptr;  // exchange buffer whose barrier this workgroup has arrived at, not yet passed
    int32_t done = 0;
    for (;;) {
        const int32_t ks = P.steps - done < P.kstep ? P.steps - done : P.kstep;
        if constexpr (STATIC) {
        for (int32_t j = 1; j <= ks; ++j) {
            // one round from buffer C (a compile-time choice, so every LDS
            // address below is a register plus a constant)
            auto round = [&](auto Cc) {
                constexpr uint32_t C = decltype(Cc)::value, NX = C == 2 ? 0 : C + 1, CL = NX == 2 ? 0 : NX + 1;
                const uint32_t *src = s_buf + C * WORDS;
                uint32_t *dst = s_buf + NX * WORDS;
                if (imp) {
                    tile_blocks<Pat, NT>(A, U, src, dst, ~defer);
                    if (tid == 0) barrier_poll(P.bar, base + nbar, P.flag);
                    __syncthreads();
                    v = 0;
                    if (tid < kMaxRing)
                        v = here ? (__hip_atomic_load(imp + gi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u) : 0u;
                    if (v) atomicOr(lds_word(s_buf + C * WORDS, home), 1u << (home & 31));
                    __syncthreads();
                    tile_blocks<Pat, NT>(A, U, src, dst, defer);
                    imp = nullptr;
                } else {
                    tile_blocks<Pat, NT>(A, U, src, dst);
                }
                if (j < ks) {
                    uint32_t *clr = s_buf + CL * WORDS;
                    if (tid < WORDS - LDS::VIRT) clr[LDS::VIRT + tid] = 0;
                    if (tid < s_rs[ks - j]) {
                        const uint4 e0 = *reinterpret_cast<const uint4 *>(s_ring + tid * 8);
                        const uint4 e1 = *reinterpret_cast<const uint4 *>(s_ring + tid * 8 + 4);
                        const uint32_t cnt = lds_bit(src, e0.x) + lds_bit(src, e0.y) + lds_bit(src, e0.z) +
                                             lds_bit(src, e0.w) + lds_bit(src, e1.x) + lds_bit(src, e1.y) +
                                             lds_bit(src, e1.z) + lds_bit(src, e1.w);
                        const uint32_t h = s_ring[kMaxRing * 8 + tid];
                        const uint32_t self = lds_bit(src, h);
                        if (here & ((cnt == 3) | (self & (cnt == 2)))) atomicOr(lds_word(dst, h), 1u << (h & 31));
                    }
                }
            };
            if (cur == 0)
                round(std::integral_constant<uint32_t, 0>{});
            else if (cur == 1)
                round(std::integral_constant<uint32_t, 1>{});
            else
                round(std::integral_constant<uint32_t, 2>{});
            __syncthreads();
            cur = cur == 2 ? 0 : cur + 1;
        }
        } else {
        for (int32_t j = 1; j <= ks; ++j) {
            const uint32_t nx = cur == 2 ? 0 : cur + 1, cl = nx == 2 ? 0 : nx + 1;
            const uint32_t *src = s_buf + cur * WORDS;
            uint32_t *dst = s_buf + nx * WORDS;
            if (imp) {
                tile_blocks<Pat, NT>(A, R, src, dst, ~defer);
                if (tid == 0) barrier_poll(P.bar, base + nbar, P.flag);
                __syncthreads();
                v = 0;
                if (tid < kMaxRing)
                    v = here ? (__hip_atomic_load(imp + gi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u) : 0u;
                if (v) atomicOr(lds_word(s_buf + cur * WORDS, home), 1u << (home & 31));
                __syncthreads();
                tile_blocks<Pat, NT>(A, R, src, dst, defer);
                imp = nullptr;
            } else if (A.nblocks == LDS::NBMAX) {
                tile_blocks<Pat, NT, true>(A, R, src, dst);
            } else {
                tile_blocks<Pat, NT>(A, R, src, dst);
            }
            if (j < ks) {
                uint32_t *clr = s_buf + cl * WORDS;
                if (tid < WORDS - LDS::VIRT) clr[LDS::VIRT + tid] = 0;
                if (tid < s_rs[ks - j]) {
                    const uint4 e0 = *reinterpret_cast<const uint4 *>(s_ring + tid * 8);
                    const uint4 e1 = *reinterpret_cast<const uint4 *>(s_ring + tid * 8 + 4);
                    const uint32_t cnt = lds_bit(src, e0.x) + lds_bit(src, e0.y) + lds_bit(src, e0.z) +
                                         lds_bit(src, e0.w) + lds_bit(src, e1.x) + lds_bit(src, e1.y) +
                                         lds_bit(src, e1.z) + lds_bit(src, e1.w);
                    const uint32_t h = s_ring[kMaxRing * 8 + tid];
                    const uint32_t self = lds_bit(src, h);
                    if (here & ((cnt == 3) | (self & (cnt == 2)))) atomicOr(lds_word(dst, h), 1u << (h & 31));
                }
            }
            __syncthreads();
            cur = nx;
        }
        }
        done += ks;
        if (done >= P.steps) break;
        // exchange: boundary cells out, ring cells in
        uint8_t *xb = (nbar & 1) ? P.a : P.b;
        const uint32_t *st = s_buf + cur * WORDS;
        for (uint32_t i = tid; i < P.nbound; i += NT) {
            const uint32_t z = P.bound[i];
            __hip_atomic_store(xb + S0 + z, (uint8_t)((st[z / NC] >> (z % NC)) & 1u), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tid < WORDS - LDS::VIRT) {
            s_buf[LDS::VIRT + tid] = 0;
            s_buf[WORDS + LDS::VIRT + tid] = 0;
            s_buf[2 * WORDS + LDS::VIRT + tid] = 0;
        }
        ++nbar;
        if (SQZ_SPLIT_EXCHANGE) {
            __builtin_amdgcn_s_waitcnt(0);  // this wave's exchange stores are complete
            __syncthreads();
            if (tid == 0) barrier_arrive(P.bar, base + nbar);
            imp = xb;  // the next round waits for the barrier after updating the other slots
        } else {
            grid_barrier(P.bar, base + nbar, P.flag);
            v = 0;
            if (tid < kMaxRing)
                v = here ? (__hip_atomic_load(xb + gi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u) : 0u;
            if (v) atomicOr(lds_word(s_buf + cur * WORDS, home), 1u << (home & 31));
            __syncthreads();
        }
    }
    // The state goes to the buffer of the step count's parity.  A tile reads an
    // exchange buffer only between the barrier that closes that exchange and its
    // own arrival at the next barrier, and reads the start buffer `a` only before
    // its first one; so only the last exchange's buffer (exchange j goes through
    // b for odd j, a for even j; `a` counts as exchange 0) may still be in use,
    // and only a store into it must wait for every tile.
    if ((uint32_t)(P.steps & 1) == (nbar & 1)) {
        ++nbar;
        grid_barrier(P.bar, base + nbar, P.flag);
    }
    // every workgroup has passed a barrier of this run, so has read the base
    if (nbar && blockIdx.x == 0 && tid == 0)
        __hip_atomic_store(P.bar + 2, base + nbar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tile_store<Pat, NT, true>(A, (P.steps & 1) ? P.b : P.a, A0, o, W, s_buf + cur * WORDS);
}

}  // namespace sqz
