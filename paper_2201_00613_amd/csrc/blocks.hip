// Block-level layouts of the comparison approaches (Section "Experimental
// Setup and Results") and block-level Squeeze storage (Section "Moving from
// Thread-level to Block-level").
//
// Blocks are the level-m subtrees: block t holds compact cells
// [t k^m, (t+1) k^m), and its cells lie in the s^m x s^m box with origin
// s^m * lambda_{r-m}(t).  Two layouts of the states:
//   lambda(omega): the expanded n x n array (row-major, holes 0); workgroups
//     run over the compact grid of blocks, so only member blocks are touched,
//     but the array still takes n^2 bytes.
//   micro-blocks: k^(r-m) blocks in compact (replica-major) order, each an
//     expanded s^m x s^m micro-fractal (row-major, holes stored as 0):
//     k^(r-m) s^(2m) bytes, the memory of the paper's block-level Squeeze.
// Both steps stage each block with a one-cell ring in LDS and update four
// positions per 32-bit word (byte-wise neighbour sums, (count|self)==3),
// masked by the micro-fractal so holes stay 0.
//
// Coarse maps come from the level-r maps: the first cell of block t is
// lambda_r(t k^m) = lambda_m(0) + s^m lambda_{r-m}(t) with lambda_m(0) inside
// [0, s^m)^2, so lambda_{r-m}(t) = floor(lambda_r(t k^m) / s^m); and a block
// (X, Y) is a member iff nu_r(X s^m + a, Y s^m + b) is not a hole for the
// member point (a, b) = lambda_m(0) of the micro-fractal, in which case it is
// block nu_r(...) / k^m.
#include <cstring>

#include "common.h"

namespace sqz {

namespace {

constexpr int kBlk = 256;
constexpr int kMaxBox = 64;     // largest block side s^m
constexpr int kMaxGroup = 128;  // blocks staged together by one workgroup

struct BlkArgs {
    MapParams P;            // level-r maps
    uint64_t nblocks;       // k^(r-m)
    uint64_t km;            // k^m
    Div64 dkm;              // division by k^m
    int32_t B, Pt, rows;    // block side, LDS pitch (4 (ceil(B/4) + 2) bytes), box rows (B + 2)
    int32_t G;              // blocks per pass
    int32_t a, b;           // lambda_m(0): a member point of the micro-fractal
    int64_t n;              // expanded side
    uint32_t off_mask, off_nb, off_org;  // LDS offsets
};

// Box layout in LDS: row 0 and row B+1 are the ring, column 3 and column B+4
// the ring, interior cell (x, y) of the block at (y + 1) * Pt + x + 4; the
// rest is zero padding.  Word w of a row covers columns 4w..4w+3, so block
// columns 4(w-1)..4(w-1)+3 when B is a multiple of 4.
__device__ __forceinline__ uint32_t box_at(const BlkArgs &A, int x, int y) { return (uint32_t)((y + 1) * A.Pt + x + 4); }

__device__ __forceinline__ void origin_of(const BlkArgs &A, uint64_t t, uint32_t &X, uint32_t &Y)
{
    uint32_t x, y;
    const uint64_t c = t * A.km;
    if (A.P.N <= 0x100000000ull)
        lam_map32(A.P, (uint32_t)c, x, y);
    else
        lam_map64(A.P, c, x, y);
    X = x / (uint32_t)A.B;
    Y = y / (uint32_t)A.B;
}

// Block index of block (X + dx, Y + dy), kHole64 when it is not a member.
__device__ __forceinline__ uint64_t block_nu(const BlkArgs &A, uint32_t X, uint32_t Y, int dx, int dy)
{
    const int64_t gx = ((int64_t)X + dx) * A.B + A.a, gy = ((int64_t)Y + dy) * A.B + A.b;
    if (gx < 0 || gy < 0 || gx >= A.n || gy >= A.n) return kHole64;
    const uint64_t c = nu_map(A.P, (int32_t)gx, (int32_t)gy);
    return c == kHole64 ? kHole64 : divq(c, A.dkm);
}

template <bool EXP>
__global__ void __launch_bounds__(kBlk) k_life_blocks(BlkArgs A, const uint8_t *__restrict__ in,
                                                      uint8_t *__restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint8_t *box = smem;  // G boxes of Pt * rows bytes
    uint8_t *mask = smem + A.off_mask;
    uint64_t *nb = reinterpret_cast<uint64_t *>(smem + A.off_nb);  // 9 per block: own index, then 8 neighbours
    uint32_t *org = reinterpret_cast<uint32_t *>(smem + A.off_org);
    const int tid = threadIdx.x, B = A.B, Pt = A.Pt, rows = A.rows, G = A.G;
    const uint32_t boxsz = (uint32_t)(Pt * rows);
    const uint64_t B2 = (uint64_t)B * (uint64_t)B;
    // zero every box (pads and absent ring cells stay 0) and build the
    // micro-fractal mask from block 0's box
    for (uint32_t i = tid; i < (uint32_t)G * boxsz; i += kBlk) box[i] = 0;
    {
        uint32_t X0, Y0;
        origin_of(A, 0, X0, Y0);
        for (uint32_t i = tid; i < boxsz; i += kBlk) mask[i] = 0;
        __syncthreads();
        for (int i = tid; i < B * B; i += kBlk) {
            const int x = i % B, y = i / B;
            mask[box_at(A, x, y)] = nu_map(A.P, (int32_t)(X0 * B + x), (int32_t)(Y0 * B + y)) != kHole64;
        }
    }
    const uint64_t passes = (A.nblocks + G - 1) / G;
    const int W4 = Pt / 4, wrow = (B + 3) / 4;  // words per box row; interior words per row
    for (uint64_t q = blockIdx.x; q < passes; q += gridDim.x) {
        const uint64_t t0 = q * (uint64_t)G;
        const int g_here = (int)((A.nblocks - t0) < (uint64_t)G ? (A.nblocks - t0) : (uint64_t)G);
        __syncthreads();  // previous pass done with LDS
        for (int j = tid; j < g_here; j += kBlk) {
            uint32_t X, Y;
            origin_of(A, t0 + j, X, Y);
            org[2 * j] = X;
            org[2 * j + 1] = Y;
        }
        if (!EXP) {
            __syncthreads();
            for (int j = tid; j < 8 * g_here; j += kBlk) {
                const int g = j / 8, d = j % 8, dd = d < 4 ? d : d + 1;
                nb[9 * g + 1 + d] = block_nu(A, org[2 * g], org[2 * g + 1], dd % 3 - 1, dd / 3 - 1);
            }
        }
        __syncthreads();
        // interior: B rows of B bytes per block
        if ((B & 3) == 0) {
            const int per = B * B / 4;
            for (int j = tid; j < g_here * per; j += kBlk) {
                const int g = j / per, w = j % per, y = (4 * w) / B, x = (4 * w) % B;
                uint32_t v;
                if (EXP)
                    v = *reinterpret_cast<const uint32_t *>(in + ((uint64_t)org[2 * g + 1] * B + y) * (uint64_t)A.n +
                                                             (uint64_t)org[2 * g] * B + x);
                else
                    v = *reinterpret_cast<const uint32_t *>(in + (t0 + g) * B2 + (uint64_t)(4 * w));
                *reinterpret_cast<uint32_t *>(box + g * boxsz + box_at(A, x, y)) = v;
            }
        } else {
            for (int j = tid; j < g_here * B * B; j += kBlk) {
                const int g = j / (B * B), i = j % (B * B), y = i / B, x = i % B;
                box[g * boxsz + box_at(A, x, y)] =
                    EXP ? in[((uint64_t)org[2 * g + 1] * B + y) * (uint64_t)A.n + (uint64_t)org[2 * g] * B + x]
                        : in[(t0 + g) * B2 + (uint64_t)i];
            }
        }
        // ring: 4B + 4 cells per block
        const int ring = 4 * B + 4;
        for (int j = tid; j < g_here * ring; j += kBlk) {
            const int g = j / ring, e = j % ring;
            int x, y;  // block-relative, -1 or B on the ring
            if (e < B + 2) {
                x = e - 1;
                y = -1;
            } else if (e < 2 * B + 4) {
                x = e - (B + 2) - 1;
                y = B;
            } else if (e < 3 * B + 4) {
                x = -1;
                y = e - (2 * B + 4);
            } else {
                x = B;
                y = e - (3 * B + 4);
            }
            uint8_t v = 0;
            if (EXP) {
                const int64_t gx = (int64_t)org[2 * g] * B + x, gy = (int64_t)org[2 * g + 1] * B + y;
                if (gx >= 0 && gy >= 0 && gx < A.n && gy < A.n) v = in[(uint64_t)gy * (uint64_t)A.n + (uint64_t)gx];
            } else {
                const int dx = x < 0 ? -1 : (x >= B ? 1 : 0), dy = y < 0 ? -1 : (y >= B ? 1 : 0);
                const int d = (dy + 1) * 3 + (dx + 1);
                const uint64_t blk = nb[9 * g + 1 + (d < 4 ? d : d - 1)];
                if (blk != kHole64) v = in[blk * B2 + (uint64_t)((y - dy * B) * B + (x - dx * B))];
            }
            box[g * boxsz + (uint32_t)((y + 1) * Pt + x + 4)] = v;
        }
        __syncthreads();
        // update: interior words of every row, masked
        for (int j = tid; j < g_here * B * wrow; j += kBlk) {
            const int g = j / (B * wrow), i = j % (B * wrow), y = i / wrow, w = 1 + i % wrow;
            const uint32_t *q32 = reinterpret_cast<const uint32_t *>(box + g * boxsz) + y * W4 + w;
            const uint32_t a0 = q32[-1], b0 = q32[0], c0 = q32[1];
            const uint32_t a1 = q32[W4 - 1], b1 = q32[W4], c1 = q32[W4 + 1];
            const uint32_t a2 = q32[2 * W4 - 1], b2 = q32[2 * W4], c2 = q32[2 * W4 + 1];
            const uint32_t cnt = b0 + __builtin_amdgcn_alignbyte(b0, a0, 3) + __builtin_amdgcn_alignbyte(c0, b0, 1) +
                                 b2 + __builtin_amdgcn_alignbyte(b2, a2, 3) + __builtin_amdgcn_alignbyte(c2, b2, 1) +
                                 __builtin_amdgcn_alignbyte(b1, a1, 3) + __builtin_amdgcn_alignbyte(c1, b1, 1);
            const uint32_t z = (cnt | b1) ^ 0x03030303u;
            const uint32_t live = (~(((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) >> 7) & 0x01010101u;
            const uint32_t res = live & reinterpret_cast<const uint32_t *>(mask)[(y + 1) * W4 + w];
            const int x0 = 4 * (w - 1);
            if ((B & 3) == 0) {
                uint8_t *dst = EXP ? out + ((uint64_t)org[2 * g + 1] * B + y) * (uint64_t)A.n + (uint64_t)org[2 * g] * B + x0
                                   : out + (t0 + g) * B2 + (uint64_t)(y * B + x0);
                *reinterpret_cast<uint32_t *>(dst) = res;
            } else {
                for (int u = 0; u < 4 && x0 + u < B; ++u) {
                    const uint8_t v = (uint8_t)(res >> (8 * u));
                    if (EXP)
                        out[((uint64_t)org[2 * g + 1] * B + y) * (uint64_t)A.n + (uint64_t)org[2 * g] * B + x0 + u] = v;
                    else
                        out[(t0 + g) * B2 + (uint64_t)(y * B + x0 + u)] = v;
                }
            }
        }
    }
}

// micro-block layout <-> compact layout
__global__ void __launch_bounds__(kBlk) k_blocks_pack(BlkArgs A, const uint8_t *__restrict__ compact,
                                                      uint8_t *__restrict__ blocks)
{
    const uint64_t B2 = (uint64_t)A.B * (uint64_t)A.B, total = A.nblocks * B2;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlk + threadIdx.x; i < total; i += (uint64_t)gridDim.x * kBlk) {
        const uint64_t t = i / B2;
        const uint32_t w = (uint32_t)(i - t * B2), x = w % (uint32_t)A.B, y = w / (uint32_t)A.B;
        uint32_t X, Y;
        origin_of(A, t, X, Y);
        const uint64_t c = nu_map(A.P, (int32_t)(X * A.B + x), (int32_t)(Y * A.B + y));
        blocks[i] = c == kHole64 ? 0 : compact[c];
    }
}

__global__ void __launch_bounds__(kBlk) k_blocks_unpack(BlkArgs A, const uint8_t *__restrict__ blocks,
                                                        uint8_t *__restrict__ compact)
{
    const uint64_t B2 = (uint64_t)A.B * (uint64_t)A.B;
    for (uint64_t c = (uint64_t)blockIdx.x * kBlk + threadIdx.x; c < A.P.N; c += (uint64_t)gridDim.x * kBlk) {
        uint32_t x, y;
        if (A.P.N <= 0x100000000ull)
            lam_map32(A.P, (uint32_t)c, x, y);
        else
            lam_map64(A.P, c, x, y);
        const uint64_t t = divq(c, A.dkm);
        compact[c] = blocks[t * B2 + (uint64_t)(y % (uint32_t)A.B) * A.B + x % (uint32_t)A.B];
    }
}

uint64_t ipow(uint64_t b, int e)
{
    uint64_t v = 1;
    for (int i = 0; i < e; ++i) v *= b;
    return v;
}

}  // namespace

// Block side s^m and validity of level m for these layouts.
sqz_status blocks_check(const FractalHost &F, int m, int64_t *side)
{
    if (m < 0 || m > F.r) return set_error(SQZ_ERR_RANGE, "block level %d outside [0, %d]", m, F.r);
    const uint64_t B = ipow((uint64_t)F.s, m);
    if (B > (uint64_t)kMaxBox)
        return set_error(SQZ_ERR_UNSUPPORTED, "block side %llu exceeds %d", (unsigned long long)B, kMaxBox);
    if (side) *side = (int64_t)B;
    return SQZ_OK;
}

static void make_args(const FractalHost &F, int m, BlkArgs &A, size_t &lds)
{
    memset(&A, 0, sizeof(A));
    A.P = F.P;
    A.B = (int32_t)ipow((uint64_t)F.s, m);
    A.km = ipow((uint64_t)F.k, m);
    A.nblocks = F.N / A.km;
    A.dkm = make_div64(A.km);
    A.Pt = 4 * ((A.B + 3) / 4 + 2);  // pads, left ring, interior words, right ring
    A.rows = A.B + 2;
    int G = 4096 / (A.B * A.B);
    A.G = G < 1 ? 1 : (G > kMaxGroup ? kMaxGroup : G);
    int64_t x0, y0;
    host_lambda(F, F.r, 0, x0, y0);
    A.a = (int32_t)(x0 % A.B);
    A.b = (int32_t)(y0 % A.B);
    A.n = F.n;
    const size_t boxsz = (size_t)A.Pt * A.rows;
    size_t off = (size_t)A.G * boxsz;
    off = (off + 15) / 16 * 16;
    A.off_mask = (uint32_t)off;
    off = (off + boxsz + 15) / 16 * 16;
    A.off_nb = (uint32_t)off;
    off += (size_t)A.G * 9 * 8;
    A.off_org = (uint32_t)off;
    off += (size_t)A.G * 2 * 4;
    lds = off;
}

uint64_t blocks_bytes(const FractalHost &F, int m)
{
    const uint64_t B = ipow((uint64_t)F.s, m);
    return F.N / ipow((uint64_t)F.k, m) * B * B;
}

static unsigned blocks_grid(uint64_t passes)
{
    uint64_t g = passes;
    if (g > 2048 * 8) g = 2048 * 8;
    return (unsigned)(g ? g : 1);
}

sqz_status launch_life_blocks(const FractalHost &F, int m, bool expanded, const uint8_t *in, uint8_t *out,
                              hipStream_t st)
{
    BlkArgs A;
    size_t lds;
    make_args(F, m, A, lds);
    const unsigned grid = blocks_grid((A.nblocks + A.G - 1) / A.G);
    if (expanded)
        hipLaunchKernelGGL(k_life_blocks<true>, dim3(grid), dim3(kBlk), lds, st, A, in, out);
    else
        hipLaunchKernelGGL(k_life_blocks<false>, dim3(grid), dim3(kBlk), lds, st, A, in, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, expanded ? "lambda_omega_step launch" : "microblock_step launch");
}

sqz_status launch_blocks_convert(const FractalHost &F, int m, bool pack, const uint8_t *src, uint8_t *dst,
                                 hipStream_t st)
{
    BlkArgs A;
    size_t lds;
    make_args(F, m, A, lds);
    const uint64_t items = pack ? blocks_bytes(F, m) : F.N;
    uint64_t g = (items + kBlk - 1) / kBlk;
    if (g > 16384) g = 16384;
    if (g == 0) g = 1;
    if (pack)
        hipLaunchKernelGGL(k_blocks_pack, dim3((unsigned)g), dim3(kBlk), 0, st, A, src, dst);
    else
        hipLaunchKernelGGL(k_blocks_unpack, dim3((unsigned)g), dim3(kBlk), 0, st, A, src, dst);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, pack ? "microblock_pack launch" : "microblock_unpack launch");
}

}  // namespace sqz
