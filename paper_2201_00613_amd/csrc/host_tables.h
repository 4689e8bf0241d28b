// Host-only part of libsqueeze: the fractal descriptor, error reporting, and
// the construction of every table the kernels read (chunked map tables,
// bit-sliced tile rings and halos, expanded-tile ring slots, bit-row tile
// borders).  Plain C++17 with no HIP dependency: it is compiled by g++ into
// the library, and by the CPU tests under AddressSanitizer and
// UndefinedBehaviorSanitizer.  The HIP sources upload what it builds.
//
// Compact storage is one value per fractal cell in the replica-major order:
// compact index c has base-k digits beta_1..beta_r (beta_mu = digit mu-1,
// least significant first) and lives at expanded coordinate
// lambda(c) = sum_mu tau(beta_mu) * s^(mu-1) (Section "Revisiting lambda").
// Every level-m subtree is therefore a contiguous range [t*k^m, (t+1)*k^m).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "squeeze.h"

namespace sqz {

constexpr uint32_t kNuHole32 = 0xFFFFFFFFu;
constexpr uint64_t kHole64 = ~0ull;
constexpr int kMaxS = 16;
constexpr int kMaxK = 256;

// ---------------------------------------------------------------------------
// Division by a run-time invariant integer (Granlund & Montgomery, "Division
// by invariant integers using multiplication", PLDI 1994, unsigned case):
// with l = ceil(log2 d) and m = floor(2^W (2^l - d) / d) + 1,
// q = (t + ((n - t) >> min(l,1))) >> max(l-1,0), t = mulhi(m, n), exact for
// every W-bit n.
// ---------------------------------------------------------------------------
struct Div32 {
    uint32_t d, m, sh1, sh2;
};
struct Div64 {
    uint64_t d, m;
    uint32_t sh1, sh2;
};

Div32 make_div32(uint32_t d);
Div64 make_div64(uint64_t d);

// ---------------------------------------------------------------------------
// Chunked look-up tables for the two maps.
//
// lambda: a chunk of CL base-k digits d (value < k^CL) maps to the packed
//   offset (x | y << 16) = sum over the chunk's levels of tau(digit) s^level.
// nu: a chunk of CN base-s digit pairs (xc, yc), both < s^CN, maps to the
//   chunk's replica digits read as a base-k number, or kNuHole32 when any
//   level's digit pair is not a replica offset (explicit hole test; the
//   paper's arithmetic hash has no hole value).
// The top chunk of each map covers the remaining r - CL*(chunks-1) levels
// and has its own table, so digits above level r never contribute.
// ---------------------------------------------------------------------------
struct MapParams {
    int32_t s, k, r, n;       // n = s^r < 2^31
    uint64_t N;               // k^r
    int32_t nlam, nnu;        // number of chunks (0 when r == 0)
    uint32_t klam, slam;      // k^CL, s^CL
    uint32_t snu, snu_top;    // s^CN, s^(top nu chunk levels)
    uint64_t knu;             // k^CN
    Div64 dklam64;
    Div32 dklam32;
    Div32 dsnu;
    const uint32_t *lam_lo, *lam_top, *nu_lo, *nu_top;  // device tables (set by the uploader)
    uint32_t ntab;            // words of the four tables, stored contiguously from lam_lo
};

// Contents of the four map tables of one level, concatenated in the order
// lam_lo, lam_top, nu_lo, nu_top; off[i] is the first entry of table i.
struct MapTables {
    std::vector<uint32_t> all;
    size_t off[4];
};

// ---------------------------------------------------------------------------
// Host-side fractal handle.
// ---------------------------------------------------------------------------
struct TileConfig;    // life_tile.hip
struct XTileConfig;   // xtile.hip
struct MfmaParams;    // mfma_maps.hip
struct BitboxConfig;  // bitbox.hip

struct FractalHost {
    int32_t s, k, r;
    int64_t n;
    uint64_t N;
    int32_t ox[kMaxK], oy[kMaxK];
    int32_t hnu[kMaxS * kMaxS];  // replica index of digit pair (x + s*y), -1 if none
    int device;
    MapParams P;                  // maps at level r
    void *d_tables;               // device memory holding the chunk tables
    // tiled stencil (patterns with a specialised kernel), built on demand
    int tile_kind;                // 0 = none
    TileConfig *tile;
    XTileConfig *xtile;           // expanded-tile kernels (any pattern), null if none
    MfmaParams *mfma;             // matrix-core map variants, null if unsupported (k > 127)
    BitboxConfig *bitbox;         // bit-row expanded tiles (dense s = 3 patterns), null if none
};

// ---------------------------------------------------------------------------
// Errors: a message per thread, returned by sqz_last_error().
// ---------------------------------------------------------------------------
sqz_status set_error(sqz_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
const char *last_error_text();

// Descriptor (s, k replica offsets, r) validation (the fractal definition of
// the Introduction): 2 <= s <= 16, 1 <= k <= s^2 distinct offsets in [0,s)^2,
// r >= 0, n = s^r < 2^31, N = k^r < 2^62.  Fills F's descriptor fields when F
// is not null.
sqz_status check_descriptor(int32_t s, int32_t k, const int32_t *offs, int32_t r, FractalHost *F);

// Scalar fields of P (its table pointers stay null) and the table contents
// for the maps at `level`.
void map_tables(const FractalHost &F, int level, MapParams &P, MapTables &T);

// Plain maps of the pattern at a given level (local coordinates): lambda as a
// digit sum, nu as a level scan (-1 for holes and points outside the box).
void host_lambda(const FractalHost &F, int level, uint64_t c, int64_t &x, int64_t &y);
int64_t host_nu(const FractalHost &F, int level, int64_t x, int64_t y);

// ---------------------------------------------------------------------------
// Bit-sliced tile tables (Section "Moving from Thread-level to Block-level"):
// a tile is a level-M subtree, a block a level-J subtree held as one LDS word.
// ---------------------------------------------------------------------------
struct TileSpec {
    int M, J;                     // tile and block levels
    int nc, box;                  // cells of a block, side of a block's box
    int ngrp;                     // adjacent-block directions a block's halo reads
    int g_dx[8], g_dy[8];
    uint32_t lds_zero, lds_virt, lds_ring2;  // LDS word indices of the special words
    int max_tile_halo, max_ring, max_steps;
};

struct TileTables {
    uint32_t nthalo = 0;          // ring-1 cells
    uint32_t ksteps = 1;          // steps one launch can take
    uint32_t ring_start[16] = {}; // slots of ring d: [ring_start[d-1], ring_start[d]), d <= max_steps
    uint32_t tstride = 0;         // ring cells loaded per tile
    uint32_t nsrc = 0;            // ring cells advanced in LDS
    uint32_t nbstride = 0;        // u32 entries per block of nbt
    std::vector<int32_t> slots;   // per ring cell: tile dx, tile dy, cell index in that tile, 0
    std::vector<uint32_t> nbt;    // per block: 16-bit LDS byte offsets of its adjacent-block words
    std::vector<uint32_t> home;   // per ring cell: LDS entry (byte offset << 16 | bit)
    std::vector<uint32_t> rsrc;   // per advanced ring cell: LDS entries of its 8 neighbours
    std::vector<uint32_t> bound;  // tile-local indices of the cells other tiles load as ring cells
};

// SQZ_ERR_UNSUPPORTED when ring 1 exceeds spec.max_tile_halo.
sqz_status tile_tables(const FractalHost &F, const TileSpec &S, TileTables &T);

// ---------------------------------------------------------------------------
// Expanded-tile tables: the level-M subtree scattered into a P-pitch box with
// a border of `border` cells filled from the eight adjacent subtrees.
// ---------------------------------------------------------------------------
struct XRingSlot {
    uint16_t pos;   // box position
    uint32_t info;  // adjacent-tile direction (0..7) << 16 | cell index in that tile
};

// Ring of one cell (border 1): member cells of the adjacent tiles that touch
// the tile, each once, in tile-cell order.
void xtile_ring_slots(const FractalHost &F, int M, uint32_t P, std::vector<XRingSlot> &out);

// Per tile cell: box position (border 1) and the 32-bit entry holding the box
// position in bits 0..15, the member neighbours inside the tile in bits
// 16..19, and per adjacent tile the number of its member cells the cell
// touches at bit field_shift[d8].
void xtile_cell_entries(const FractalHost &F, int M, uint32_t P, const int field_shift[8],
                        std::vector<uint16_t> &lam, std::vector<uint32_t> &ent);

// Multi-step form with a K-cell border: ring slots by Chebyshev layer
// (start[d] = first slot of layer d+1), box positions of the tile's cells and
// the membership of the tile's own box positions (P x rows bytes).
void xtile_layer_tables(const FractalHost &F, int M, int K, uint32_t P, uint32_t rows,
                        std::vector<XRingSlot> &ring, std::vector<uint32_t> &start, std::vector<uint16_t> &lam,
                        std::vector<uint8_t> &mem);

// ---------------------------------------------------------------------------
// Bit-row tile tables (patterns of side 3, level-1 blocks of one byte): grid
// positions of a tile's blocks, the border blocks of the adjacent tiles, and
// membership of every box position as bit rows.
// ---------------------------------------------------------------------------
struct BitboxSpec {
    int M;             // tile level
    int border;        // border blocks on each side
    int grid_pitch;    // bytes per row of the block grid
    int rows, words;   // rows and 32-bit words per row of the membership box
};

void bitbox_tables(const FractalHost &F, const BitboxSpec &S, std::vector<uint16_t> &bpos,
                   std::vector<uint32_t> &ring, std::vector<uint32_t> &member);

}  // namespace sqz
