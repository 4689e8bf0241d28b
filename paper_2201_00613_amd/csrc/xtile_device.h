// Expanded-tile kernels: block-level Squeeze (Section "Moving from
// Thread-level to Block-level") for any NBB pattern, for Life and for the
// explicit diffusion update.
//
// A tile is a level-M subtree: compact range [t K^M, (t+1) K^M).  Its cells
// are scattered into an on-chip copy of the tile's s^M x s^M expanded box,
// with a one-cell ring around it (pitch P = s^M + 2), through a tile-invariant
// table of local lambda positions.  The ring holds the few cells of adjacent
// tiles that touch the tile; their compact addresses are the adjacent tiles'
// bases (eight coarse nu at level r-M, evaluated once per tile) plus a
// tile-invariant cell index.  Every cell then reads its eight neighbours at
// fixed offsets in LDS (holes hold 0 and are never written) and writes its
// result in compact order, so global reads and writes are coalesced.
//
// The grid is persistent: each workgroup keeps the tables in LDS and walks a
// contiguous run of tiles, so the neighbouring tiles whose ring cells it reads
// were just loaded into (or are about to be loaded into) its XCD's L2.
//
// Diffusion (the PDE application named in the Introduction): u' = u + a (S -
// deg u), S the sum of the member neighbours' values, deg their count (no flux
// through holes or the box edge), evaluated in binary32 in a fixed order.
// bfloat16 storage keeps delta = u - offset with a caller-chosen offset (the
// mean, which the update conserves); the update is linear, so it runs on delta
// directly, accumulates in binary32 and rounds to bfloat16 either to nearest
// even or stochastically with 16 counter-hash bits per (seed, step, cell).
#pragma once

#include "common.h"

namespace sqz {

constexpr int kXBlock = 256;
constexpr size_t kXLdsBudget = 48 * 1024;

struct XArgs {
    uint64_t ntiles;
    uint32_t KM, P, R, B;  // cells per tile, row pitch (multiple of 4), ring slots, box side
    uint32_t off_val, off_res, off_mem, off_lam, off_rpos, off_rinfo, off_nbase;
    uint32_t vec;  // 1 when a tile is a whole number of 16-byte vectors
    // multi-step tiles: border of K cells, `rows` box rows; ring slots of layer d
    // (Chebyshev distance d from the tile's box) are [ring_start[d-1], ring_start[d])
    uint32_t K, rows;
    uint32_t ring_start[4];
    const uint16_t *lam;
    const uint8_t *mem_in;
    const uint32_t *ent;  // per cell: lambda position | member-neighbour fields << 16 (diffusion)
    const uint16_t *rpos;
    const uint32_t *rinfo;
    MapParams Pc;
};

struct XOp {
    float coef;
    uint32_t rounding;  // sqz_rounding
    uint64_t seed, step;
};

// kWaves: the one-step kernel's minimum waves per SIMD (register budget; the
// diffusion kernels keep every lane's sixteen cell entries in registers, and
// the measured best is four waves for binary32, five for bfloat16 storage).
struct XLife {
    using G = uint8_t;
    using L = uint8_t;
    static constexpr bool kMem = false;
    static constexpr bool kSwar = true;  // row-wise SIMD-within-a-register update
    static constexpr int kVec = 16;
    static constexpr int kWaves = 1;
};
struct XDiffF32 {
    using G = float;
    using L = float;
    static constexpr bool kMem = true;
    static constexpr bool kSwar = false;
    static constexpr int kVec = 4;
    static constexpr int kWaves = 4;
};
struct XDiffBF16 {
    using G = uint16_t;  // bfloat16 bits of delta
    using L = float;
    static constexpr bool kMem = true;
    static constexpr bool kSwar = false;
    static constexpr int kVec = 8;
    static constexpr int kWaves = 5;
};

__device__ __forceinline__ uint8_t to_lds(uint8_t v) { return v; }
__device__ __forceinline__ float to_lds(float v) { return v; }
__device__ __forceinline__ float to_lds(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// 16 pseudo-random bits per (seed, step, cell): the "lowbias32" integer
// finaliser (C. Wellons, hash-prospector, 2018) of a Weyl combination of the
// counters.  32-bit arithmetic keeps the per-cell cost and register use low.
__device__ __forceinline__ uint32_t rand16(uint64_t seed, uint64_t step, uint64_t cell)
{
    uint32_t x = (uint32_t)cell ^ ((uint32_t)(cell >> 32) * 0x85EBCA6Bu);
    x += (uint32_t)seed * 0x9E3779B9u + (uint32_t)(seed >> 32) + (uint32_t)step * 0x7FEB352Du;
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x >> 16;
}

// binary32 -> bfloat16 bits: nearest-even, or stochastic (add 16 random bits
// below the kept mantissa, truncate).
__device__ __forceinline__ uint16_t to_bf16(float u, uint32_t rounding, uint32_t r16)
{
    uint32_t b = __float_as_uint(u);
    b += rounding == SQZ_ROUND_STOCHASTIC ? r16 : 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// u' = u + a (S - deg u) in binary32 (S summed in a fixed order), stored as
// binary32 or as bfloat16 bits.
template <class Op>
__device__ __forceinline__ typename Op::G diff_finish(float S, float c, uint32_t deg, const XOp &op, uint64_t gcell)
{
    const float u = fmaf(op.coef, fmaf(-(float)deg, c, S), c);
    if constexpr (sizeof(typename Op::G) == 4)
        return u;
    else
        return to_bf16(u, op.rounding, op.rounding == SQZ_ROUND_STOCHASTIC ? rand16(op.seed, op.step, gcell) : 0u);
}

template <class Op>
__device__ __forceinline__ typename Op::G cell_update(const typename Op::L *s_val, const uint8_t *s_mem, uint32_t p,
                                                      uint32_t P, const XOp &op, uint64_t gcell)
{
    using L = typename Op::L;
    const L *b = s_val + (p - P - 1);
    const L n0 = b[0], n1 = b[1], n2 = b[2], n3 = b[P], c = b[P + 1], n4 = b[P + 2];
    const L n5 = b[2 * P], n6 = b[2 * P + 1], n7 = b[2 * P + 2];
    if constexpr (!Op::kMem) {
        const uint32_t cnt = (uint32_t)n0 + n1 + n2 + n3 + n4 + n5 + n6 + n7;
        return (typename Op::G)(cnt == 3 || (c && cnt == 2));
    } else {
        const uint8_t *m = s_mem + (p - P - 1);
        const uint32_t deg = (uint32_t)m[0] + m[1] + m[2] + m[P] + m[P + 2] + m[2 * P] + m[2 * P + 1] + m[2 * P + 2];
        const float S = ((((((n0 + n1) + n2) + n3) + n4) + n5) + n6) + n7;
        return diff_finish<Op>(S, c, deg, op, gcell);
    }
}

// Member-neighbour count of a tile cell without a membership array.  The
// cell's entry holds its lambda position in bits 0..15, the number of its
// member neighbours inside the tile in bits 16..19, and for each adjacent tile
// the number of that tile's member cells it touches: two bits for the four
// side tiles (up to three cells), one bit for the four corner tiles.  Which
// adjacent tiles exist varies per tile; lo / hi select the fields of those
// present, with weights 1 and 2.
struct DegMask {
    uint32_t lo, hi;
};
// field of adjacent tile d8 (d8 = index of (dx, dy) in row-major order of the
// 3 x 3 neighbourhood without its centre)
__host__ __device__ constexpr int deg_field(int d8)
{
    return d8 == 1 ? 20 : d8 == 3 ? 22 : d8 == 4 ? 24 : d8 == 6 ? 26 : d8 == 0 ? 28 : d8 == 2 ? 29 : d8 == 5 ? 30 : 31;
}
__host__ __device__ constexpr bool deg_side(int d8) { return d8 == 1 || d8 == 3 || d8 == 4 || d8 == 6; }

__device__ __forceinline__ DegMask deg_mask(const uint64_t *nbase)
{
    DegMask m{0u, 0u};
#pragma unroll
    for (int d = 0; d < 8; ++d)
        if (nbase[d] != kHole64) {
            m.lo |= 1u << deg_field(d);
            if (deg_side(d)) m.hi |= 2u << deg_field(d);
        }
    return m;
}

template <class Op>
__device__ __forceinline__ typename Op::G diff_update(const float *s_val, uint32_t e, uint32_t P, DegMask dm,
                                                      const XOp &op, uint64_t gcell)
{
    const float *b = s_val + ((e & 0xFFFFu) - P - 1);
    const float n0 = b[0], n1 = b[1], n2 = b[2], n3 = b[P], c = b[P + 1], n4 = b[P + 2];
    const float n5 = b[2 * P], n6 = b[2 * P + 1], n7 = b[2 * P + 2];
    const uint32_t deg = ((e >> 16) & 15u) + __popc(e & dm.lo) + 2u * __popc(e & dm.hi);
    const float S = ((((((n0 + n1) + n2) + n3) + n4) + n5) + n6) + n7;
    return diff_finish<Op>(S, c, deg, op, gcell);
}

// LDS carve-up of the expanded tile (offsets in XArgs).
template <class Op>
struct XLds {
    typename Op::L *val;
    uint8_t *res;  // row-update results (Life)
    uint16_t *lam, *rpos;
    uint32_t *rinfo;
    uint64_t *nbase;
    __device__ XLds(unsigned char *smem, const XArgs &A)
        : val(reinterpret_cast<typename Op::L *>(smem + A.off_val)), res(smem + A.off_res),
          lam(reinterpret_cast<uint16_t *>(smem + A.off_lam)), rpos(reinterpret_cast<uint16_t *>(smem + A.off_rpos)),
          rinfo(reinterpret_cast<uint32_t *>(smem + A.off_rinfo)), nbase(reinterpret_cast<uint64_t *>(smem + A.off_nbase))
    {
    }
};

// Zero the expanded box and copy the tile-invariant tables into LDS.
template <class Op>
__device__ __forceinline__ void xtile_setup(const XArgs &A, const XLds<Op> &S)
{
    const uint32_t tid = threadIdx.x, PP = A.P * A.P;
    for (uint32_t i = tid; i < PP; i += kXBlock) {
        S.val[i] = (typename Op::L)0;
    }
    if constexpr (Op::kSwar) {  // the 16 bytes on either side of the box: row updates read them
        uint32_t *before = reinterpret_cast<uint32_t *>(S.val) - 4;
        uint32_t *after = reinterpret_cast<uint32_t *>(S.val + PP);
        if (tid < 4) before[tid] = 0;
        else if (tid < 8) after[tid - 4] = 0;
    }
    if constexpr (!Op::kMem)
        for (uint32_t i = tid; i < A.KM; i += kXBlock) S.lam[i] = A.lam[i];
    for (uint32_t i = tid; i < A.R; i += kXBlock) {
        S.rpos[i] = A.rpos[i];
        S.rinfo[i] = A.rinfo[i];
    }
}

// Box position of tile cell l: the LDS lambda table (Life) or the cell's
// entry (diffusion).
template <class Op>
__device__ __forceinline__ uint32_t xt_pos(const XArgs &A, const XLds<Op> &S, uint32_t l)
{
    if constexpr (Op::kMem)
        return A.ent[l] & 0xFFFFu;
    else
        return S.lam[l];
}

// One tile t: scatter, ring, update.  Starts with a barrier (tables ready and
// the previous tile's LDS reads done).  Called by every lane.
template <class Op, int PT>
__device__ __forceinline__ void xtile_body(const XArgs &A, const typename Op::G *__restrict__ in,
                                           typename Op::G *__restrict__ out, uint64_t t, const XOp &op,
                                           const XLds<Op> &S)
{
    using G = typename Op::G;
    using L = typename Op::L;
    constexpr int VEC = Op::kVec;
    const uint32_t P = PT ? (uint32_t)PT : A.P;
    const uint32_t KM = A.KM, R = A.R, tid = threadIdx.x;
    __syncthreads();
    // adjacent tiles' first cells (eight coarse nu of this tile's coarse cell)
    if (tid < 8) {
        const int d = tid < 4 ? (int)tid : (int)tid + 1;
        uint32_t X, Y;
        if (A.Pc.N <= 0x100000000ull)
            lam_map32(A.Pc, (uint32_t)t, X, Y);
        else
            lam_map64(A.Pc, t, X, Y);
        const uint64_t nt = nu_map(A.Pc, (int32_t)X + d % 3 - 1, (int32_t)Y + d / 3 - 1);
        S.nbase[tid] = nt == kHole64 ? kHole64 : nt * KM;
    }
    // scatter the tile's cells into the expanded box
    const G *src = in + t * KM;
    if (A.vec) {
        for (uint32_t v = tid; v < KM / VEC; v += kXBlock) {
            const uint4 q = *reinterpret_cast<const uint4 *>(src + (size_t)v * VEC);
            const G *e = reinterpret_cast<const G *>(&q);
#pragma unroll
            for (int i = 0; i < VEC; ++i) S.val[xt_pos<Op>(A, S, v * VEC + i)] = to_lds(e[i]);
        }
    } else {
        for (uint32_t l = tid; l < KM; l += kXBlock) S.val[xt_pos<Op>(A, S, l)] = to_lds(src[l]);
    }
    __syncthreads();
    // the ring: cells of adjacent tiles that touch this one
    for (uint32_t j = tid; j < R; j += kXBlock) {
        const uint32_t info = S.rinfo[j];
        const uint64_t nb = S.nbase[info >> 16];
        L v = (L)0;
        if (nb != kHole64) v = to_lds(in[nb + (info & 0xFFFFu)]);
        S.val[S.rpos[j]] = v;
    }
    __syncthreads();
    // update every cell, results in compact order
    G *dst = out + t * KM;
    const uint64_t gbase = t * KM;
    if constexpr (Op::kMem) {
        const DegMask dm = deg_mask(S.nbase);
        for (uint32_t l = tid; l < KM; l += kXBlock) dst[l] = diff_update<Op>(S.val, A.ent[l], P, dm, op, gbase + l);
    } else if (A.vec) {
        for (uint32_t v = tid; v < KM / VEC; v += kXBlock) {
            uint4 q;
            G *e = reinterpret_cast<G *>(&q);
#pragma unroll
            for (int i = 0; i < VEC; ++i)
                e[i] = cell_update<Op>(S.val, nullptr, S.lam[v * VEC + i], P, op, gbase + v * VEC + i);
            *reinterpret_cast<uint4 *>(dst + (size_t)v * VEC) = q;
        }
    } else {
        for (uint32_t l = tid; l < KM; l += kXBlock) dst[l] = cell_update<Op>(S.val, nullptr, S.lam[l], P, op, gbase + l);
    }
}

// Bases of the eight tiles adjacent to tile t (eight coarse nu at level r-M),
// written by lanes 0..7 to dst[0..7]; kHole64 where there is no tile.
__device__ __forceinline__ void xtile_bases(const XArgs &A, uint64_t t, uint64_t *dst)
{
    const uint32_t tid = threadIdx.x;
    if (tid < 8) {
        const int d = tid < 4 ? (int)tid : (int)tid + 1;
        uint32_t X, Y;
        if (A.Pc.N <= 0x100000000ull)
            lam_map32(A.Pc, (uint32_t)t, X, Y);
        else
            lam_map64(A.Pc, t, X, Y);
        const uint64_t nt = nu_map(A.Pc, (int32_t)X + d % 3 - 1, (int32_t)Y + d / 3 - 1);
        dst[tid] = nt == kHole64 ? kHole64 : nt * A.KM;
    }
}

// Tiles [t0, t1) with software pipelining: while tile t is updated from LDS,
// the cells and ring cells of tile t+1 are already in flight into registers.
// Cell l of a tile is handled by lane l mod 256 (cells k*256 + lane), so the
// lanes of one wave touch one compact level-2 block: nearby expanded positions,
// few LDS bank conflicts, and coalesced global accesses.  KPL >= KM/256 and
// RPL >= R/256 bound the per-lane registers; FULL means KM == KPL * 256 (no
// per-cell bounds test).  Called by every lane.
template <class Op, int PT, int KPL, int RPL, bool FULL = false>
__device__ __forceinline__ void xtile_run(const XArgs &A, const typename Op::G *__restrict__ in,
                                          typename Op::G *__restrict__ out, uint64_t t0, uint64_t t1, const XOp &op,
                                          const XLds<Op> &S)
{
    using G = typename Op::G;
    using L = typename Op::L;
    const uint32_t P = PT ? (uint32_t)PT : A.P;
    const uint32_t KM = A.KM, R = A.R, tid = threadIdx.x;
    if (t0 >= t1) return;
    G cur[KPL];
    L rv[RPL];
    // diffusion: the entries of this lane's cells, the same for every tile
    uint32_t ent[Op::kMem ? KPL : 1];
    if constexpr (Op::kMem) {
#pragma unroll
        for (int k = 0; k < KPL; ++k) {
            const uint32_t l = (uint32_t)k * 256 + tid;
            ent[k] = (FULL || l < KM) ? A.ent[l] : 0u;
        }
    }
    __syncthreads();  // tables and the previous work's LDS reads are done
    xtile_bases(A, t0, S.nbase + 8 * (t0 & 1));
    __syncthreads();
    // prologue: tile t0's cells and ring into registers
    {
        const G *src = in + t0 * KM;
        const uint64_t *nb = S.nbase + 8 * (t0 & 1);
#pragma unroll
        for (int k = 0; k < KPL; ++k) {
            const uint32_t l = (uint32_t)k * 256 + tid;
            if (FULL || l < KM) cur[k] = src[l];
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t j = (uint32_t)k * 256 + tid;
            rv[k] = (L)0;
            if (j < R) {
                const uint32_t info = S.rinfo[j];
                const uint64_t b = nb[info >> 16];
                if (b != kHole64) rv[k] = to_lds(in[b + (info & 0xFFFFu)]);
            }
        }
    }
    for (uint64_t t = t0; t < t1; ++t) {
        __syncthreads();  // previous tile's update no longer reads LDS
#pragma unroll
        for (int k = 0; k < KPL; ++k) {
            const uint32_t l = (uint32_t)k * 256 + tid;
            if (FULL || l < KM) {
                if constexpr (Op::kMem)
                    S.val[ent[k] & 0xFFFFu] = to_lds(cur[k]);
                else
                    S.val[S.lam[l]] = to_lds(cur[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t j = (uint32_t)k * 256 + tid;
            if (j < R) S.val[S.rpos[j]] = rv[k];
        }
        const bool more = t + 1 < t1;
        if (more) xtile_bases(A, t + 1, S.nbase + 8 * ((t + 1) & 1));
        __syncthreads();
        if (more) {  // issue tile t+1's loads before updating tile t
            const G *src = in + (t + 1) * KM;
            const uint64_t *nb = S.nbase + 8 * ((t + 1) & 1);
#pragma unroll
            for (int k = 0; k < KPL; ++k) {
                const uint32_t l = (uint32_t)k * 256 + tid;
                if (FULL || l < KM) cur[k] = src[l];
            }
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const uint32_t j = (uint32_t)k * 256 + tid;
                rv[k] = (L)0;
                if (j < R) {
                    const uint32_t info = S.rinfo[j];
                    const uint64_t b = nb[info >> 16];
                    if (b != kHole64) rv[k] = to_lds(in[b + (info & 0xFFFFu)]);
                }
            }
        }
        G *dst = out + t * KM;
        const uint64_t gbase = t * KM;
        if constexpr (Op::kSwar) {
            // Life on whole box rows, four positions per 32-bit word: byte-wise
            // neighbour sums of the three rows shifted by one byte either way,
            // then (count | self) == 3 per byte.  Ring and holes hold 0.
            const uint32_t W4 = P / 4, nrow = A.B;
            const uint32_t *v32 = reinterpret_cast<const uint32_t *>(S.val);
            uint32_t *r32 = reinterpret_cast<uint32_t *>(S.res);
            for (uint32_t idx = tid; idx < nrow * W4; idx += kXBlock) {
                const uint32_t y = 1 + idx / W4, w = idx - (y - 1) * W4;
                const uint32_t *q = v32 + (y - 1) * W4 + w;  // q[-1] and the word after the box are padding
                const uint32_t a0 = q[-1], b0 = q[0], c0 = q[1];
                const uint32_t a1 = q[W4 - 1], b1 = q[W4], c1 = q[W4 + 1];
                const uint32_t a2 = q[2 * W4 - 1], b2 = q[2 * W4], c2 = q[2 * W4 + 1];
                const uint32_t cnt = b0 + __builtin_amdgcn_alignbyte(b0, a0, 3) + __builtin_amdgcn_alignbyte(c0, b0, 1) +
                                     b2 + __builtin_amdgcn_alignbyte(b2, a2, 3) + __builtin_amdgcn_alignbyte(c2, b2, 1) +
                                     __builtin_amdgcn_alignbyte(b1, a1, 3) + __builtin_amdgcn_alignbyte(c1, b1, 1);
                const uint32_t z = (cnt | b1) ^ 0x03030303u;
                r32[y * W4 + w] = (~(((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) >> 7) & 0x01010101u;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < KPL; ++k) {
                const uint32_t l = (uint32_t)k * 256 + tid;
                if (FULL || l < KM) dst[l] = S.res[S.lam[l]];
            }
        } else {
            const DegMask dm = deg_mask(S.nbase + 8 * (t & 1));
#pragma unroll
            for (int k = 0; k < KPL; ++k) {
                const uint32_t l = (uint32_t)k * 256 + tid;
                if (FULL || l < KM) dst[l] = diff_update<Op>(S.val, ent[k], P, dm, op, gbase + l);
            }
        }
    }
}

// Host-side configuration of the expanded tiles of one fractal.
struct XTileConfig {
    int M;
    uint32_t KM, B, P, R;
    uint64_t ntiles;
    void *d_tab;
    XArgs base;  // tables; LDS offsets are filled per operation
    size_t lds_life, lds_diff;
    unsigned grid_life, grid_diff, grid_diff16;  // persistent grids (diff16: bfloat16 storage)
    void *d_coarse;
    // multi-step form (K steps per launch; K = 0: none)
    uint32_t K;
    void *d_tabk;
    XArgs kbase;
    size_t ldsk_life, ldsk_diff;
    unsigned gridk_life, gridk_diff;
};

// LDS layout: values, row results (Life), lambda table (Life), ring tables,
// 2 x 8 bases.  Diffusion keeps its cell entries in registers or reads them
// from global memory, so its box needs no membership array.
inline size_t xt_align16(size_t v) { return (v + 15) & ~(size_t)15; }
inline size_t xt_layout(uint32_t P, uint32_t KM, uint32_t R, size_t val_bytes, bool diff, bool swar, XArgs *A)
{
    const size_t box = (size_t)P * P * val_bytes;
    const size_t off_val = 16;  // padding on both sides: row updates read one word past each end
    size_t off = xt_align16(off_val + box + 16);
    const size_t off_res = off;
    if (swar) off = xt_align16(off + (size_t)P * P);
    const size_t off_lam = off;
    if (!diff) off = xt_align16(off + (size_t)KM * 2);  // diffusion keeps cell entries in registers
    const size_t off_rpos = off;
    off = xt_align16(off + (size_t)R * 2);
    const size_t off_rinfo = off;
    off = xt_align16(off + (size_t)R * 4);
    const size_t off_nbase = off;
    off += 16 * 8;  // two sets of eight adjacent-tile bases (double-buffered)
    if (A) {
        A->off_val = (uint32_t)off_val;
        A->off_res = (uint32_t)off_res;
        A->off_lam = (uint32_t)off_lam;
        A->off_rpos = (uint32_t)off_rpos;
        A->off_rinfo = (uint32_t)off_rinfo;
        A->off_nbase = (uint32_t)off_nbase;
    }
    return off;
}

// LDS layout of the multi-step form: values (Life: two boxes), membership,
// lambda table, ring tables, 2 x 8 bases.  Boxes are P x rows with 16 zero
// bytes on both sides (row updates read one word past each end).
inline size_t xt_layoutK(uint32_t P, uint32_t rows, uint32_t KM, uint32_t R, size_t val_bytes, bool life, XArgs *A)
{
    const size_t box = (size_t)P * rows;
    const size_t off_val = 16;
    size_t off = xt_align16(off_val + box * val_bytes + 16);
    const size_t off_res = off + 16;
    if (life) off = xt_align16(off_res + box + 16);
    const size_t off_mem = off;
    off = xt_align16(off + box);
    const size_t off_lam = off;
    off = xt_align16(off + (size_t)KM * 2);
    const size_t off_rpos = off;
    off = xt_align16(off + (size_t)R * 2);
    const size_t off_rinfo = off;
    off = xt_align16(off + (size_t)R * 4);
    const size_t off_nbase = off;
    off += 16 * 8;
    if (A) {
        A->off_val = (uint32_t)off_val;
        A->off_res = (uint32_t)off_res;
        A->off_mem = (uint32_t)off_mem;
        A->off_lam = (uint32_t)off_lam;
        A->off_rpos = (uint32_t)off_rpos;
        A->off_rinfo = (uint32_t)off_rinfo;
        A->off_nbase = (uint32_t)off_nbase;
    }
    return off;
}

// Zero both boxes (with their pads) and the membership box, then copy the
// tile-invariant tables into LDS (membership of the tile's own cells included).
template <class Op>
__device__ __forceinline__ void xtile_setupK(const XArgs &A, unsigned char *smem)
{
    const uint32_t tid = threadIdx.x, box = A.P * A.rows;
    const uint32_t end = Op::kSwar ? A.off_res + box + 16 : A.off_val + box * (uint32_t)sizeof(typename Op::L) + 16;
    for (uint32_t i = tid; i < end / 4; i += kXBlock) reinterpret_cast<uint32_t *>(smem)[i] = 0;
    uint8_t *mem = smem + A.off_mem;
    for (uint32_t i = tid; i < box; i += kXBlock) mem[i] = A.mem_in[i];
    uint16_t *lam = reinterpret_cast<uint16_t *>(smem + A.off_lam);
    for (uint32_t i = tid; i < A.KM; i += kXBlock) lam[i] = A.lam[i];
    uint16_t *rpos = reinterpret_cast<uint16_t *>(smem + A.off_rpos);
    uint32_t *rinfo = reinterpret_cast<uint32_t *>(smem + A.off_rinfo);
    for (uint32_t i = tid; i < A.R; i += kXBlock) {
        rpos[i] = A.rpos[i];
        rinfo[i] = A.rinfo[i];
    }
}

// Life on box rows 1..rows-2, four positions per word, masked by membership.
__device__ __forceinline__ void xt_life_rows(const uint8_t *src, uint8_t *dst, const uint8_t *mem, uint32_t P,
                                             uint32_t rows)
{
    const uint32_t W4 = P / 4, n = (rows - 2) * W4;
    const uint32_t *v32 = reinterpret_cast<const uint32_t *>(src);
    const uint32_t *m32 = reinterpret_cast<const uint32_t *>(mem);
    uint32_t *r32 = reinterpret_cast<uint32_t *>(dst);
    for (uint32_t idx = threadIdx.x; idx < n; idx += kXBlock) {
        const uint32_t y = 1 + idx / W4, w = idx - (y - 1) * W4;
        const uint32_t *q = v32 + (y - 1) * W4 + w;
        const uint32_t a0 = q[-1], b0 = q[0], c0 = q[1];
        const uint32_t a1 = q[W4 - 1], b1 = q[W4], c1 = q[W4 + 1];
        const uint32_t a2 = q[2 * W4 - 1], b2 = q[2 * W4], c2 = q[2 * W4 + 1];
        const uint32_t cnt = b0 + __builtin_amdgcn_alignbyte(b0, a0, 3) + __builtin_amdgcn_alignbyte(c0, b0, 1) +
                             b2 + __builtin_amdgcn_alignbyte(b2, a2, 3) + __builtin_amdgcn_alignbyte(c2, b2, 1) +
                             __builtin_amdgcn_alignbyte(b1, a1, 3) + __builtin_amdgcn_alignbyte(c1, b1, 1);
        const uint32_t z = (cnt | b1) ^ 0x03030303u;
        const uint32_t live = (~(((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) >> 7) & 0x01010101u;
        r32[y * W4 + w] = live & m32[y * W4 + w];
    }
}

// K steps of every tile in [t0, t1), software-pipelined as xtile_run.  The
// box has a border of K cells; all member cells of layers 1..K are loaded
// with the tile (their membership, which depends on whether the adjacent tile
// exists, goes into the membership box).  Round j is exact on the tile and on
// layers 1..K-j, which is all that round j+1 reads.  Life: whole rows per
// round, two boxes alternating.  Diffusion: the cells of the tile and of
// layers 1..K-j, results held in registers until every lane has read the
// round's inputs; intermediate states are rounded to the storage type exactly
// as a one-step launch stores them.
template <class Op, int PT, int KPL, int RPL, int K>
__device__ __forceinline__ void xtile_runK(const XArgs &A, const typename Op::G *__restrict__ in,
                                           typename Op::G *__restrict__ out, uint64_t t0, uint64_t t1, const XOp &op,
                                           unsigned char *smem)
{
    using G = typename Op::G;
    using L = typename Op::L;
    const uint32_t P = PT ? (uint32_t)PT : A.P;
    const uint32_t KM = A.KM, R = A.R, tid = threadIdx.x;
    L *val = reinterpret_cast<L *>(smem + A.off_val);
    uint8_t *res = smem + A.off_res;
    uint8_t *mem = smem + A.off_mem;
    const uint16_t *lam = reinterpret_cast<const uint16_t *>(smem + A.off_lam);
    const uint16_t *rpos = reinterpret_cast<const uint16_t *>(smem + A.off_rpos);
    const uint32_t *rinfo = reinterpret_cast<const uint32_t *>(smem + A.off_rinfo);
    uint64_t *nbase = reinterpret_cast<uint64_t *>(smem + A.off_nbase);
    if (t0 >= t1) return;
    G cur[KPL];
    L rv[RPL];
    bool rm[RPL];
    __syncthreads();
    xtile_bases(A, t0, nbase + 8 * (t0 & 1));
    __syncthreads();
    auto fetch = [&](uint64_t t) {
        const G *src = in + t * KM;
        const uint64_t *nb = nbase + 8 * (t & 1);
#pragma unroll
        for (int k = 0; k < KPL; ++k) {
            const uint32_t l = (uint32_t)k * 256 + tid;
            if (l < KM) cur[k] = src[l];
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t j = (uint32_t)k * 256 + tid;
            rv[k] = (L)0;
            rm[k] = false;
            if (j < R) {
                const uint32_t info = rinfo[j];
                const uint64_t b = nb[info >> 16];
                if (b != kHole64) {
                    rv[k] = to_lds(in[b + (info & 0xFFFFu)]);
                    rm[k] = true;
                }
            }
        }
    };
    fetch(t0);
    for (uint64_t t = t0; t < t1; ++t) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KPL; ++k) {
            const uint32_t l = (uint32_t)k * 256 + tid;
            if (l < KM) val[lam[l]] = to_lds(cur[k]);
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t j = (uint32_t)k * 256 + tid;
            if (j < R) {
                val[rpos[j]] = rv[k];
                mem[rpos[j]] = rm[k];
            }
        }
        const uint64_t *nbt = nbase + 8 * (t & 1);
        const bool more = t + 1 < t1;
        if (more) xtile_bases(A, t + 1, nbase + 8 * ((t + 1) & 1));
        __syncthreads();
        if (more) fetch(t + 1);
        G *dst = out + t * KM;
        const uint64_t gbase = t * KM;
        if constexpr (Op::kSwar) {
            uint8_t *a = reinterpret_cast<uint8_t *>(val), *b = res;
#pragma unroll
            for (int j = 1; j <= K; ++j) {
                xt_life_rows(a, b, mem, P, A.rows);
                __syncthreads();
                uint8_t *c = a;
                a = b;
                b = c;
            }
#pragma unroll
            for (int k = 0; k < KPL; ++k) {
                const uint32_t l = (uint32_t)k * 256 + tid;
                if (l < KM) dst[l] = a[lam[l]];
            }
        } else {
#pragma unroll
            for (int j = 1; j <= K; ++j) {
                XOp oj = op;
                oj.step = op.step + (uint64_t)(j - 1);
                G nv[KPL];
#pragma unroll
                for (int k = 0; k < KPL; ++k) {
                    const uint32_t l = (uint32_t)k * 256 + tid;
                    if (l < KM) nv[k] = cell_update<Op>(val, mem, lam[l], P, oj, gbase + l);
                }
                if (j == K) {
#pragma unroll
                    for (int k = 0; k < KPL; ++k) {
                        const uint32_t l = (uint32_t)k * 256 + tid;
                        if (l < KM) dst[l] = nv[k];
                    }
                } else {
                    const uint32_t nring = A.ring_start[K - j];
                    G rn[RPL];
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        const uint32_t jj = (uint32_t)k * 256 + tid;
                        if (jj < nring) {
                            const uint32_t info = rinfo[jj];
                            const uint64_t b = nbt[info >> 16];
                            rn[k] = cell_update<Op>(val, mem, rpos[jj], P, oj, b + (info & 0xFFFFu));
                        }
                    }
                    __syncthreads();  // every lane has read the round's inputs
#pragma unroll
                    for (int k = 0; k < KPL; ++k) {
                        const uint32_t l = (uint32_t)k * 256 + tid;
                        if (l < KM) val[lam[l]] = to_lds(nv[k]);
                    }
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        const uint32_t jj = (uint32_t)k * 256 + tid;
                        if (jj < nring && mem[rpos[jj]]) val[rpos[jj]] = to_lds(rn[k]);
                    }
                    __syncthreads();
                }
            }
        }
    }
}

}  // namespace sqz
