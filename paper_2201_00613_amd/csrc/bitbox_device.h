// Block-level Squeeze (Section "Moving from Thread-level to Block-level")
// for Life on dense patterns of side s = 3 with at most 8 replicas (the
// Sierpinski carpet): the level-M subtree of a tile is expanded on chip into
// a box of bit rows, one bit per position, and Life runs on whole 32-bit row
// words.
//
// Tile  = a level-M subtree (M <= 5): compact cells [t k^M, (t+1) k^M), a
//         3^M x 3^M region of the expanded plane.
// Block = a level-1 subtree: k <= 8 consecutive compact cells in one 3 x 3
//         box, held as one byte of bits (bit j = replica j).
// Box   = the tile's blocks plus a border four blocks (twelve cells) wide
//         from the eight adjacent tiles, as bit rows: row y, word w = columns
//         32w .. 32w+31.  With a twelve-cell border one launch could take up
//         to twelve steps (each step invalidates one more cell along the box
//         edge); it takes up to ten, as the bit-sliced tiles do.
//
// Per tile: (A) each block's eight bytes are packed to one byte of bits and
// placed in a block grid (one byte per block position, tile-invariant
// positions); the border blocks come from the adjacent tiles, whose bases
// are eight coarse nu per tile.  (B) Each 32-bit row word is assembled from
// twelve consecutive grid bytes: the row's three bits of each block are cut
// out of four bytes at a time and packed together.  (C) K Life rounds on the
// row words, bit-sliced with full adders: a lane owns one word column of
// ten consecutive rows and slides a window over them; new states are
// masked by the tile-invariant membership of each position and by whether
// the adjacent tile it lies in exists.  (D) Each block's byte is read back
// from three rows and unpacked to eight bytes.
#pragma once

#include "common.h"
#include "tile_device.h"

namespace sqz {

struct PatCarpet {  // Sierpinski carpet, replicas row by row
    static constexpr int S = 3, K = 8;
    static constexpr int OX[8] = {0, 1, 2, 0, 2, 0, 1, 2};
    static constexpr int OY[8] = {0, 0, 0, 1, 1, 2, 2, 2};
};

constexpr int kBxBorder = 4;                 // border blocks on each side
constexpr int kBxBC = 3 * kBxBorder;         // border cells on each side
constexpr int kBxMMax = 5;                   // tile level: 3^5 + 24 = 267 columns
// Rows are kBxW words with no pad between them: columns 267 .. 287 are
// always zero (outside every box, masked by membership), so word 8's right
// neighbour (word 0 of the next row) and word 0's left neighbour (word 8 of
// the row before) only ever shift zeros or masked columns into the box.
constexpr int kBxW = 9;                      // row words (288 columns)
constexpr int kBxP = kBxW;                   // row pitch in words
constexpr int kBxSR = 10;                    // rows of one lane's strip
constexpr int kBxStrips = 27;                // strips: 27 x 10 rows >= 267
constexpr int kBxLanes = kBxW * kBxStrips;   // lanes with a word column (243)
constexpr int kBxRows = kBxStrips * kBxSR;   // box rows (270); rows past the box stay zero
// a zero word, a zero guard row above and below, and a zero word after it (read as the
// right neighbour of the guard row's last word)
constexpr int kBxBuf = 2 + (kBxRows + 2) * kBxP;
// LDS word of row y (-1 .. kBxRows), word w (-1 .. 9; -1 and 9 only at the buffer's ends or as
// the zero columns of the adjacent row)
__host__ __device__ constexpr int bx_at(int y, int w) { return 1 + (y + 1) * kBxP + w; }
constexpr int kBxGR = 81 + 2 * kBxBorder;    // block-grid rows (and columns): 3^4 + 2 * 4
constexpr int kBxGP = 100;                   // bytes per block-grid row (a row word reads 16 bytes from byte 84)
constexpr int kBxMaxSteps = 10;              // Life steps per launch (<= kBxBC)
constexpr int kBxThreads = 256;
constexpr int kBxMaxBlocks = 4096;           // k^(M-1) <= 8^4
static_assert(kBxGR * kBxGP <= kBxBuf * 4, "the block grid lives in the second row buffer");
static_assert(kBxLanes <= kBxThreads && kBxRows >= 3 * kBxGR && 32 * kBxW > 3 * kBxGR, "box fits the lanes");
static_assert(2 * kBxBuf * 4 + 9 * 8 + 4 <= 20 * 1024, "eight workgroups per CU");
static_assert(kBxMaxSteps <= kBxBC, "a step per border cell");
static_assert(kBxGR * kBxGP < (1 << 14), "ring slots hold the grid byte in 14 bits");

struct BitboxConfig {
    int M;
    uint32_t tile;    // k^M cells
    uint32_t nblk;    // k^(M-1) blocks
    uint32_t side;    // 3^M
    uint32_t nring;   // border blocks that can exist
    uint64_t ntiles;  // k^(r-M)
    uint16_t *d_bpos;    // [nblk] grid position of each block: x | y << 7
    uint32_t *d_ring;    // [nring] grid byte | direction << 14 | block index in that tile << 18
    uint32_t *d_member;  // [kBxRows][kBxW] membership of every box position, adjacent tiles present
    MapParams Pc;        // maps at the coarse level r-M
    void *d_coarse;
    unsigned grid;
};

struct BitboxArgs {
    uint64_t ntiles;
    uint32_t tile, nblk, side, nring;
    const uint16_t *bpos;
    const uint32_t *ring;
    const uint32_t *member;
    MapParams Pc;
};

inline BitboxArgs bitbox_args(const FractalHost &F)
{
    const BitboxConfig *C = F.bitbox;
    BitboxArgs A;
    A.ntiles = C->ntiles;
    A.tile = C->tile;
    A.nblk = C->nblk;
    A.side = C->side;
    A.nring = C->nring;
    A.bpos = C->d_bpos;
    A.ring = C->d_ring;
    A.member = C->d_member;
    A.Pc = C->Pc;
    return A;
}

template <class Pat>
__host__ __device__ constexpr int replica_at(int x, int y)
{
    for (int j = 0; j < Pat::K; ++j)
        if (Pat::OX[j] == x && Pat::OY[j] == y) return j;
    return -1;
}

// Row Q of four blocks (one byte each): bit x of byte i = position (x, Q) of block i.
template <class Pat, int Q, int X = 0>
__device__ __forceinline__ uint32_t row_field(uint32_t d)
{
    if constexpr (X == 3) {
        return 0u;
    } else {
        constexpr int j = replica_at<Pat>(X, Q);
        uint32_t v = 0;
        if constexpr (j >= X)
            v = (d >> (j - X)) & (0x01010101u << X);
        else if constexpr (j >= 0)
            v = (d << (X - j)) & (0x01010101u << X);
        return v | row_field<Pat, Q, X + 1>(d);
    }
}

// Four 3-bit fields, one per byte -> twelve consecutive bits.
__device__ __forceinline__ uint32_t compact12(uint32_t f)
{
    const uint32_t t = f | (f >> 5);
    return (t & 0x3Fu) | ((t >> 10) & 0xFC0u);
}

// Row word (cells 32w .. 32w+31 of box row 3R + Q) from twelve grid bytes
// a[0..2] = blocks C0 .. C0+11, C0 = floor(32w / 3), dl = 32w - 3 C0.
template <class Pat, int Q>
__device__ __forceinline__ uint32_t bx_rowword(const uint32_t (&a)[3], uint32_t dl)
{
    const uint32_t c0 = compact12(row_field<Pat, Q>(a[0])), c1 = compact12(row_field<Pat, Q>(a[1])),
                   c2 = compact12(row_field<Pat, Q>(a[2]));
    return __builtin_amdgcn_alignbit(c2 >> 8, c0 | (c1 << 12) | (c2 << 24), dl);
}

// Byte of a block from its three rows (bits 0..2 of r[q] = positions x = 0..2).
template <class Pat, int J = 0>
__device__ __forceinline__ uint32_t block_byte(const uint32_t (&r)[3])
{
    if constexpr (J == Pat::K) {
        return 0u;
    } else {
        constexpr int x = Pat::OX[J], y = Pat::OY[J];
        return (((r[y] >> x) & 1u) << J) | block_byte<Pat, J + 1>(r);
    }
}

// Columns [lo, hi) of the box that fall in word w, as a bit mask.
__device__ __forceinline__ uint32_t col_mask(int lo, int hi, int w)
{
    const int a = max(lo - 32 * w, 0), b = min(hi - 32 * w, 32);
    if (b <= a) return 0u;
    const uint32_t top = b == 32 ? 0xFFFFFFFFu : ((1u << b) - 1u);
    return top & ~((1u << a) - 1u);
}

// Life on one row word from three rows (each: the word and its two neighbours
// in the row).  Sums by full adders: the row above and below contribute
// three cells each (sum s3 + 2 c3), the row itself two (s2 + 2 c2).
struct BxRow {
    uint32_t s3, c3, s2, c2, c;
};

__device__ __forceinline__ BxRow bx_row(const uint32_t *p)
{
    const uint32_t L = p[-1], C = p[0], R = p[1];
    const uint32_t W = __builtin_amdgcn_alignbit(C, L, 31), E = __builtin_amdgcn_alignbit(R, C, 1);
    BxRow v;
    v.s3 = W ^ C ^ E;
    v.c3 = (W & C) | (E & (W ^ C));
    v.s2 = W ^ E;
    v.c2 = W & E;
    v.c = C;
    return v;
}

__device__ __forceinline__ uint32_t bx_life(const BxRow &u, const BxRow &m, const BxRow &d)
{
    const uint32_t x1 = u.s3 ^ m.s2 ^ d.s3, k1 = (u.s3 & m.s2) | (d.s3 & (u.s3 ^ m.s2));
    // count = x1 + 2 (c3 above + c2 + c3 below + k1): 2 or 3 iff exactly one of the four carries
    const uint32_t one = (u.c3 ^ m.c2 ^ d.c3 ^ k1) & ~((u.c3 & m.c2) | (d.c3 & k1));
    return one & (x1 | m.c);
}

// One tile, K steps (phases A to D).  LDS: s_buf = two row buffers of kBxBuf
// words (the block grid lives in the second), s_nb = nine u64, s_ex = one
// word.  Called by every lane of a workgroup of kBxThreads lanes.
template <class Pat, int K>
__device__ __forceinline__ void bitbox_tile(const BitboxArgs &A, const uint8_t *__restrict__ in,
                                            uint8_t *__restrict__ out, uint64_t t, uint32_t (*s_buf)[kBxBuf],
                                            uint64_t *s_nb, uint32_t *s_ex_p)
{
    uint32_t &s_ex = *s_ex_p;
    const uint32_t tid = threadIdx.x;
    // word column and strip of rows kBxSR ls .. kBxSR ls + kBxSR - 1 (lanes past kBxLanes idle in phase C)
    const bool act = tid < (uint32_t)kBxLanes;
    const int lw = act ? (int)(tid % kBxW) : 0, ls = act ? (int)(tid / kBxW) : 0;
    uint8_t *const G = reinterpret_cast<uint8_t *>(s_buf[1]);
    const int side = (int)A.side;
    const uint32_t mL = col_mask(0, kBxBC, lw), mC = col_mask(kBxBC, kBxBC + side, lw),
                   mR = col_mask(kBxBC + side, 2 * kBxBC + side, lw);
    {
        const uint64_t base = t * A.tile;
        // membership of this lane's words with the adjacent tiles present (tile-invariant table)
        uint32_t eff[kBxSR];
#pragma unroll
        for (int r = 0; r < kBxSR; ++r) eff[r] = act ? A.member[(kBxSR * ls + r) * kBxW + lw] : 0u;
        if (tid < 64) {
            bool here = false;
            if (tid < 9) {
                uint32_t X, Y;
                if (A.Pc.N <= 0x100000000ull)
                    lam_map32(A.Pc, (uint32_t)t, X, Y);
                else
                    lam_map64(A.Pc, t, X, Y);
                const uint64_t nt =
                    nu_map(A.Pc, (int32_t)X + (int32_t)(tid % 3) - 1, (int32_t)Y + (int32_t)(tid / 3) - 1);
                s_nb[tid] = nt == kHole64 ? kHole64 : nt * A.tile;
                here = nt != kHole64;
            }
            const uint64_t m = __ballot(here);
            if (tid == 0) s_ex = (uint32_t)m;
        }
        for (uint32_t i = tid; i < (uint32_t)kBxBuf; i += kBxThreads) {
            s_buf[0][i] = 0;
            s_buf[1][i] = 0;
        }
        __syncthreads();

        // (A) the tile's blocks and the border blocks into the grid
#pragma unroll 4
        for (uint32_t b = tid; b < A.nblk; b += kBxThreads) {
            const uint2 d = *reinterpret_cast<const uint2 *>(in + base + 8ull * b);
            const uint32_t p = A.bpos[b];
            G[(p >> 7) * kBxGP + (p & 127u)] = (uint8_t)pack8(d.x, d.y);
        }
        for (uint32_t i = tid; i < A.nring; i += kBxThreads) {
            const uint32_t slot = A.ring[i];
            const uint64_t nb = s_nb[(slot >> 14) & 15u];
            if (nb != kHole64) {
                const uint2 d = *reinterpret_cast<const uint2 *>(in + nb + 8ull * (slot >> 18));
                G[slot & 0x3FFFu] = (uint8_t)pack8(d.x, d.y);
            }
        }
        const uint32_t ex = s_ex;
        __syncthreads();

        // (B) row words from the grid: unit (block row R, word w) makes rows 3R .. 3R+2
        for (uint32_t u = tid; u < (uint32_t)(kBxGR * kBxW); u += kBxThreads) {
            const uint32_t R = u / kBxW, w = u - R * kBxW;
            const uint32_t C0 = 32 * w / 3, dl = 32 * w - 3 * C0, C0a = C0 & ~3u, o = C0 - C0a;
            const uint32_t *g = reinterpret_cast<const uint32_t *>(G + R * kBxGP + C0a);
            const uint32_t g0 = g[0], g1 = g[1], g2 = g[2], g3 = g[3];
            const uint32_t a[3] = {__builtin_amdgcn_alignbyte(g1, g0, o), __builtin_amdgcn_alignbyte(g2, g1, o),
                                   __builtin_amdgcn_alignbyte(g3, g2, o)};
            s_buf[0][bx_at(3 * R + 0, w)] = bx_rowword<Pat, 0>(a, dl);
            s_buf[0][bx_at(3 * R + 1, w)] = bx_rowword<Pat, 1>(a, dl);
            s_buf[0][bx_at(3 * R + 2, w)] = bx_rowword<Pat, 2>(a, dl);
        }
#pragma unroll
        for (int r = 0; r < kBxSR; ++r) {
            const int y = kBxSR * ls + r, ry = y < kBxBC ? 0 : (y < kBxBC + side ? 1 : 2);
            const uint32_t e3 = ex >> (3 * ry);
            eff[r] &= ((e3 & 1u) ? mL : 0u) | ((e3 & 2u) ? mC : 0u) | ((e3 & 4u) ? mR : 0u);
        }
        __syncthreads();

        // (C) K rounds; lane: word lw of rows kBxSR ls .. kBxSR ls + kBxSR - 1, sliding over one
        // row more on either side
#pragma unroll 1
        for (int j = 1; j <= K; ++j) {
            const uint32_t *src = s_buf[(j - 1) & 1];
            uint32_t *dst = s_buf[j & 1];
            if (act) {
                BxRow up = bx_row(src + bx_at(kBxSR * ls - 1, lw)), mid = bx_row(src + bx_at(kBxSR * ls, lw));
#pragma unroll
                for (int r = 0; r < kBxSR; ++r) {
                    const BxRow dn = bx_row(src + bx_at(kBxSR * ls + r + 1, lw));
                    dst[bx_at(kBxSR * ls + r, lw)] = bx_life(up, mid, dn) & eff[r];
                    up = mid;
                    mid = dn;
                }
            }
            if (tid <= (uint32_t)kBxP) dst[tid] = 0u;  // the zero word and the guard row above row 0
            __syncthreads();
        }

        // (D) blocks back to bytes
        const uint32_t *fin = s_buf[K & 1];
#pragma unroll 4
        for (uint32_t b = tid; b < A.nblk; b += kBxThreads) {
            const uint32_t p = A.bpos[b];
            const uint32_t col = 3 * (p & 127u), row = 3 * (p >> 7), wi = col >> 5, sh = col & 31u;
            uint32_t r3[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const uint32_t *rp = fin + bx_at((int)(row + q), (int)wi);
                r3[q] = __builtin_amdgcn_alignbit(rp[1], rp[0], sh) & 7u;
            }
            const uint32_t v = block_byte<Pat>(r3);
            uint2 o2;
            o2.x = spread4(v & 15u);
            o2.y = spread4(v >> 4);
            *reinterpret_cast<uint2 *>(out + base + 8ull * b) = o2;
        }
        __syncthreads();
    }
}

}  // namespace sqz
