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
#include <string.h>

#include <vector>

#include "common.h"

namespace sqz {

namespace {

constexpr int kXBlock = 256;
constexpr size_t kXLdsBudget = 48 * 1024;

struct XArgs {
    uint64_t ntiles;
    uint32_t KM, P, R;
    uint32_t off_mem, off_lam, off_rpos, off_rinfo, off_nbase;
    uint32_t vec;  // 1 when a tile is a whole number of 16-byte vectors
    const uint16_t *lam;
    const uint8_t *mem_in;
    const uint16_t *rpos;
    const uint32_t *rinfo;
    MapParams Pc;
};

struct XOp {
    float coef;
    uint32_t rounding;  // sqz_rounding
    uint64_t seed, step;
};

struct XLife {
    using G = uint8_t;
    using L = uint8_t;
    static constexpr bool kMem = false;
    static constexpr int kVec = 16;
};
struct XDiffF32 {
    using G = float;
    using L = float;
    static constexpr bool kMem = true;
    static constexpr int kVec = 4;
};
struct XDiffBF16 {
    using G = uint16_t;  // bfloat16 bits of delta
    using L = float;
    static constexpr bool kMem = true;
    static constexpr int kVec = 8;
};

__device__ __forceinline__ uint8_t to_lds(uint8_t v) { return v; }
__device__ __forceinline__ float to_lds(float v) { return v; }
__device__ __forceinline__ float to_lds(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// 16 pseudo-random bits per (seed, step, cell): SplitMix64's finaliser on a
// Weyl combination of the three counters.
__device__ __forceinline__ uint32_t rand16(uint64_t seed, uint64_t step, uint64_t cell)
{
    uint64_t z = seed + (step + 1) * 0x9E3779B97F4A7C15ull + (cell + 1) * 0xD1B54A32D192ED03ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)((z ^ (z >> 31)) >> 48);
}

// binary32 -> bfloat16 bits: nearest-even, or stochastic (add 16 random bits
// below the kept mantissa, truncate).
__device__ __forceinline__ uint16_t to_bf16(float u, uint32_t rounding, uint32_t r16)
{
    uint32_t b = __float_as_uint(u);
    b += rounding == SQZ_ROUND_STOCHASTIC ? r16 : 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
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
        const float u = fmaf(op.coef, fmaf(-(float)deg, c, S), c);
        if constexpr (sizeof(typename Op::G) == 4)
            return u;
        else
            return to_bf16(u, op.rounding, op.rounding == SQZ_ROUND_STOCHASTIC ? rand16(op.seed, op.step, gcell) : 0u);
    }
}

template <class Op, int PT>
__global__ void __launch_bounds__(kXBlock) k_xtile(XArgs A, const typename Op::G *__restrict__ in,
                                                   typename Op::G *__restrict__ out, XOp op)
{
    using G = typename Op::G;
    using L = typename Op::L;
    constexpr int VEC = Op::kVec;
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t P = PT ? (uint32_t)PT : A.P;
    const uint32_t PP = P * P, KM = A.KM, R = A.R;
    L *s_val = reinterpret_cast<L *>(smem);
    uint8_t *s_mem = smem + A.off_mem;
    uint16_t *s_lam = reinterpret_cast<uint16_t *>(smem + A.off_lam);
    uint16_t *s_rpos = reinterpret_cast<uint16_t *>(smem + A.off_rpos);
    uint32_t *s_rinfo = reinterpret_cast<uint32_t *>(smem + A.off_rinfo);
    uint64_t *s_nbase = reinterpret_cast<uint64_t *>(smem + A.off_nbase);
    const uint32_t tid = threadIdx.x;

    for (uint32_t i = tid; i < PP; i += kXBlock) {
        s_val[i] = (L)0;
        if constexpr (Op::kMem) s_mem[i] = A.mem_in[i];
    }
    for (uint32_t i = tid; i < KM; i += kXBlock) s_lam[i] = A.lam[i];
    for (uint32_t i = tid; i < R; i += kXBlock) {
        s_rpos[i] = A.rpos[i];
        s_rinfo[i] = A.rinfo[i];
    }

    const uint64_t chunk = (A.ntiles + gridDim.x - 1) / gridDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t t1 = t0 + chunk < A.ntiles ? t0 + chunk : A.ntiles;
    for (uint64_t t = t0; t < t1; ++t) {
        __syncthreads();  // tables ready / previous tile's reads of LDS done
        // adjacent tiles' first cells (eight coarse nu of this tile's coarse cell)
        if (tid < 8) {
            const int d = tid < 4 ? (int)tid : (int)tid + 1;
            uint32_t X, Y;
            if (A.Pc.N <= 0x100000000ull)
                lam_map32(A.Pc, (uint32_t)t, X, Y);
            else
                lam_map64(A.Pc, t, X, Y);
            const uint64_t nt = nu_map(A.Pc, (int32_t)X + d % 3 - 1, (int32_t)Y + d / 3 - 1);
            s_nbase[tid] = nt == kHole64 ? kHole64 : nt * KM;
        }
        // scatter the tile's cells into the expanded box
        const G *src = in + t * KM;
        if (A.vec) {
            for (uint32_t v = tid; v < KM / VEC; v += kXBlock) {
                const uint4 q = *reinterpret_cast<const uint4 *>(src + (size_t)v * VEC);
                const G *e = reinterpret_cast<const G *>(&q);
#pragma unroll
                for (int i = 0; i < VEC; ++i) s_val[s_lam[v * VEC + i]] = to_lds(e[i]);
            }
        } else {
            for (uint32_t l = tid; l < KM; l += kXBlock) s_val[s_lam[l]] = to_lds(src[l]);
        }
        __syncthreads();
        // the ring: cells of adjacent tiles that touch this one
        for (uint32_t j = tid; j < R; j += kXBlock) {
            const uint32_t info = s_rinfo[j];
            const uint64_t nb = s_nbase[info >> 16];
            L v = (L)0;
            if (nb != kHole64) v = to_lds(in[nb + (info & 0xFFFFu)]);
            s_val[s_rpos[j]] = v;
            if constexpr (Op::kMem) s_mem[s_rpos[j]] = nb != kHole64;
        }
        __syncthreads();
        // update every cell, results in compact order
        G *dst = out + t * KM;
        const uint64_t gbase = t * KM;
        if (A.vec) {
            for (uint32_t v = tid; v < KM / VEC; v += kXBlock) {
                uint4 q;
                G *e = reinterpret_cast<G *>(&q);
#pragma unroll
                for (int i = 0; i < VEC; ++i)
                    e[i] = cell_update<Op>(s_val, s_mem, s_lam[v * VEC + i], P, op, gbase + v * VEC + i);
                *reinterpret_cast<uint4 *>(dst + (size_t)v * VEC) = q;
            }
        } else {
            for (uint32_t l = tid; l < KM; l += kXBlock) dst[l] = cell_update<Op>(s_val, s_mem, s_lam[l], P, op, gbase + l);
        }
    }
}

// ---------------------------------------------------------------------------
// Thread-level diffusion (one lambda and eight nu per cell), for patterns or
// levels without an expanded tile.
// ---------------------------------------------------------------------------
template <class Op>
__global__ void __launch_bounds__(256) k_diffuse_cell(MapParams P, const typename Op::G *__restrict__ in,
                                                      typename Op::G *__restrict__ out, XOp op)
{
    for (uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x; c < P.N; c += (uint64_t)gridDim.x * 256) {
        uint32_t x, y;
        if (P.N <= 0x100000000ull)
            lam_map32(P, (uint32_t)c, x, y);
        else
            lam_map64(P, c, x, y);
        float nv[8];
        uint32_t deg = 0;
#pragma unroll
        for (int j = 0, k = 0; j < 9; ++j) {
            if (j == 4) continue;
            const uint64_t q = nu_map(P, (int32_t)x + j % 3 - 1, (int32_t)y + j / 3 - 1);
            nv[k++] = q == kHole64 ? 0.0f : to_lds(in[q]);
            deg += q != kHole64;
        }
        const float cv = to_lds(in[c]);
        const float S = ((((((nv[0] + nv[1]) + nv[2]) + nv[3]) + nv[4]) + nv[5]) + nv[6]) + nv[7];
        const float u = fmaf(op.coef, fmaf(-(float)deg, cv, S), cv);
        if constexpr (sizeof(typename Op::G) == 4)
            out[c] = u;
        else
            out[c] = to_bf16(u, op.rounding, op.rounding == SQZ_ROUND_STOCHASTIC ? rand16(op.seed, op.step, c) : 0u);
    }
}

// ---------------------------------------------------------------------------
// Binary64 mass, deterministic: fixed grid, per-lane strided sums, LDS tree
// per workgroup, then one workgroup folds the partials.  N * offset is added
// once at the end.
// ---------------------------------------------------------------------------
constexpr int kMassGrid = 1024;

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

template <class G>
__global__ void __launch_bounds__(256) k_mass_partial(const G *__restrict__ u, uint64_t N, double *__restrict__ part)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (uint64_t)kMassGrid * 256)
        acc += (double)to_lds(u[i]);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_mass_final(double *part, uint64_t N, double offset)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < kMassGrid; i += 256) acc += part[1 + i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[0] = s + (double)N * offset;
}

__global__ void __launch_bounds__(256) k_encode_bf16(const float *__restrict__ u, float offset, uint16_t *__restrict__ b,
                                                     uint64_t N)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (uint64_t)gridDim.x * 256)
        b[i] = to_bf16(u[i] - offset, SQZ_ROUND_NEAREST_EVEN, 0u);
}

__global__ void __launch_bounds__(256) k_decode_bf16(const uint16_t *__restrict__ b, float offset, float *__restrict__ u,
                                                     uint64_t N)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (uint64_t)gridDim.x * 256)
        u[i] = offset + to_lds(b[i]);
}

unsigned grid_for(uint64_t count)
{
    uint64_t g = (count + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct XTileConfig {
    int M;
    uint32_t KM, B, P, R;
    uint64_t ntiles;
    void *d_tab;
    XArgs base;  // tables and offsets (LDS offsets for the diffusion layout)
    size_t lds_life, lds_diff;
    unsigned grid_life, grid_diff;
    void *d_coarse;
};

static size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// LDS layout: values, membership bytes (diffusion), lambda table, ring tables, 8 bases.
static size_t xt_layout(uint32_t P, uint32_t KM, uint32_t R, size_t val_bytes, bool mem, XArgs *A)
{
    size_t off = align16((size_t)P * P * val_bytes);
    const size_t off_mem = off;
    if (mem) off = align16(off + (size_t)P * P);
    const size_t off_lam = off;
    off = align16(off + (size_t)KM * 2);
    const size_t off_rpos = off;
    off = align16(off + (size_t)R * 2);
    const size_t off_rinfo = off;
    off = align16(off + (size_t)R * 4);
    const size_t off_nbase = off;
    off += 8 * 8;
    if (A) {
        A->off_mem = (uint32_t)off_mem;
        A->off_lam = (uint32_t)off_lam;
        A->off_rpos = (uint32_t)off_rpos;
        A->off_rinfo = (uint32_t)off_rinfo;
        A->off_nbase = (uint32_t)off_nbase;
    }
    return off;
}

struct RingSlot {
    uint16_t pos;
    uint32_t info;
};

static void ring_slots(const FractalHost &F, int M, uint32_t P, std::vector<RingSlot> &out)
{
    int64_t side = 1;
    uint64_t KM = 1;
    for (int i = 0; i < M; ++i) {
        side *= F.s;
        KM *= F.k;
    }
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
                out.push_back(RingSlot{(uint16_t)pos, (d8 << 16) | (uint32_t)j});
            }
    }
}

template <class Op, int PT>
static unsigned occupancy_grid(size_t lds, uint64_t ntiles, int device)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_xtile<Op, PT>, kXBlock, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) cus = prop.multiProcessorCount;
    uint64_t g = (uint64_t)cus * (uint64_t)per_cu;
    if (g > ntiles) g = ntiles;
    return (unsigned)(g < 1 ? 1 : g);
}

sqz_status xtile_prepare(FractalHost &F)
{
    F.xtile = nullptr;
    if (F.r < 1) return SQZ_OK;
    // the largest level whose expanded tile fits the LDS budget in binary32
    int M = F.r < 12 ? F.r : 12;
    std::vector<RingSlot> ring;
    for (; M >= 1; --M) {
        uint64_t B = 1, KM = 1;
        for (int i = 0; i < M; ++i) {
            B *= F.s;
            KM *= F.k;
        }
        const uint64_t P = B + 2;
        if (P * P > 65535 || KM > 65535) continue;
        if (xt_layout((uint32_t)P, (uint32_t)KM, 0, 4, true, nullptr) > kXLdsBudget) continue;
        ring_slots(F, M, (uint32_t)P, ring);
        if (xt_layout((uint32_t)P, (uint32_t)KM, (uint32_t)ring.size(), 4, true, nullptr) <= kXLdsBudget) break;
    }
    if (M < 1) return SQZ_OK;  // no expanded tile for this pattern
    XTileConfig *X = new XTileConfig();
    X->M = M;
    X->B = 1;
    X->KM = 1;
    for (int i = 0; i < M; ++i) {
        X->B *= F.s;
        X->KM *= F.k;
    }
    X->P = X->B + 2;
    X->R = (uint32_t)ring.size();
    const uint32_t P = X->P, KM = X->KM, R = X->R;

    // tables: lambda positions, interior membership, ring positions, ring info
    std::vector<uint16_t> lam(KM);
    std::vector<uint8_t> mem((size_t)P * P, 0);
    for (uint32_t c = 0; c < KM; ++c) {
        int64_t x, y;
        host_lambda(F, M, c, x, y);
        lam[c] = (uint16_t)((y + 1) * P + (x + 1));
        mem[lam[c]] = 1;
    }
    const size_t o_lam = 0, o_mem = align16(o_lam + KM * 2), o_rpos = align16(o_mem + (size_t)P * P),
                 o_rinfo = align16(o_rpos + (size_t)R * 2), total = align16(o_rinfo + (size_t)R * 4 + 4);
    std::vector<uint8_t> blob(total, 0);
    memcpy(blob.data() + o_lam, lam.data(), KM * 2);
    memcpy(blob.data() + o_mem, mem.data(), (size_t)P * P);
    for (uint32_t j = 0; j < R; ++j) {
        memcpy(blob.data() + o_rpos + 2 * j, &ring[j].pos, 2);
        memcpy(blob.data() + o_rinfo + 4 * j, &ring[j].info, 4);
    }
    hipError_t e = hipMalloc(&X->d_tab, total);
    if (e == hipSuccess) e = hipMemcpy(X->d_tab, blob.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete X;
        return hip_error(e, "expanded-tile tables");
    }
    sqz_status st = build_map_params(F, F.r - M, X->base.Pc, &X->d_coarse);
    if (st != SQZ_OK) {
        (void)hipFree(X->d_tab);
        delete X;
        return st;
    }
    X->ntiles = X->base.Pc.N;
    const uint8_t *b = (const uint8_t *)X->d_tab;
    X->base.ntiles = X->ntiles;
    X->base.KM = KM;
    X->base.P = P;
    X->base.R = R;
    X->base.lam = (const uint16_t *)(b + o_lam);
    X->base.mem_in = b + o_mem;
    X->base.rpos = (const uint16_t *)(b + o_rpos);
    X->base.rinfo = (const uint32_t *)(b + o_rinfo);
    X->lds_life = xt_layout(P, KM, R, 1, false, nullptr);
    X->lds_diff = xt_layout(P, KM, R, 4, true, nullptr);
    X->grid_life = occupancy_grid<XLife, 0>(X->lds_life, X->ntiles, F.device);
    X->grid_diff = occupancy_grid<XDiffF32, 0>(X->lds_diff, X->ntiles, F.device);
    F.xtile = X;
    return SQZ_OK;
}

void xtile_release(FractalHost &F)
{
    if (!F.xtile) return;
    (void)hipFree(F.xtile->d_tab);
    (void)hipFree(F.xtile->d_coarse);
    delete F.xtile;
    F.xtile = nullptr;
}

int32_t xtile_level_of(const FractalHost &F) { return F.xtile ? F.xtile->M : 0; }

template <class Op>
static sqz_status launch_x(const FractalHost &F, const void *in, void *out, const XOp &op, hipStream_t st)
{
    const XTileConfig *X = F.xtile;
    XArgs A = X->base;
    const bool life = !Op::kMem;
    const size_t lds = xt_layout(X->P, X->KM, X->R, sizeof(typename Op::L), Op::kMem, &A);
    A.vec = ((X->KM * sizeof(typename Op::G)) % 16 == 0 && !(((uintptr_t)in | (uintptr_t)out) & 15)) ? 1u : 0u;
    const unsigned grid = life ? X->grid_life : X->grid_diff;
    using G = typename Op::G;
    const G *i = (const G *)in;
    G *o = (G *)out;
    switch (X->P) {
    case 66: hipLaunchKernelGGL((k_xtile<Op, 66>), dim3(grid), dim3(kXBlock), lds, st, A, i, o, op); break;
    case 83: hipLaunchKernelGGL((k_xtile<Op, 83>), dim3(grid), dim3(kXBlock), lds, st, A, i, o, op); break;
    default: hipLaunchKernelGGL((k_xtile<Op, 0>), dim3(grid), dim3(kXBlock), lds, st, A, i, o, op); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "expanded-tile launch");
}

sqz_status launch_life_xtile(const FractalHost &F, const uint8_t *in, uint8_t *out, hipStream_t st)
{
    if (!F.xtile) return set_error(SQZ_ERR_UNSUPPORTED, "no expanded tile for this fractal");
    XOp op{};
    return launch_x<XLife>(F, in, out, op, st);
}

sqz_status launch_diffuse(const FractalHost &F, int dtype, float coef, int rounding, uint64_t seed, uint64_t step,
                          const void *in, void *out, int use_tile, hipStream_t st)
{
    XOp op;
    op.coef = coef;
    op.rounding = (uint32_t)rounding;
    op.seed = seed;
    op.step = step;
    if (use_tile && F.xtile)
        return dtype == SQZ_F32 ? launch_x<XDiffF32>(F, in, out, op, st) : launch_x<XDiffBF16>(F, in, out, op, st);
    if (dtype == SQZ_F32)
        hipLaunchKernelGGL(k_diffuse_cell<XDiffF32>, dim3(grid_for(F.N)), dim3(256), 0, st, F.P, (const float *)in,
                           (float *)out, op);
    else
        hipLaunchKernelGGL(k_diffuse_cell<XDiffBF16>, dim3(grid_for(F.N)), dim3(256), 0, st, F.P,
                           (const uint16_t *)in, (uint16_t *)out, op);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "diffusion (cell) launch");
}

sqz_status launch_mass(const FractalHost &F, int dtype, const void *u, double offset, double *work, hipStream_t st)
{
    if (dtype == SQZ_F32)
        hipLaunchKernelGGL(k_mass_partial<float>, dim3(kMassGrid), dim3(256), 0, st, (const float *)u, F.N, work + 1);
    else
        hipLaunchKernelGGL(k_mass_partial<uint16_t>, dim3(kMassGrid), dim3(256), 0, st, (const uint16_t *)u, F.N,
                           work + 1);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(256), 0, st, work, F.N, offset);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "mass launch");
}

sqz_status launch_bf16_convert(const FractalHost &F, int encode, const float *u, float offset, uint16_t *b,
                               hipStream_t st)
{
    if (encode)
        hipLaunchKernelGGL(k_encode_bf16, dim3(grid_for(F.N)), dim3(256), 0, st, u, offset, b, F.N);
    else
        hipLaunchKernelGGL(k_decode_bf16, dim3(grid_for(F.N)), dim3(256), 0, st, (const uint16_t *)b, offset,
                           (float *)u, F.N);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "bf16 conversion launch");
}

int mass_grid() { return kMassGrid; }

}  // namespace sqz
