// Thread-level kernels: the two space maps, the seeded starts and the
// thread-level Squeeze Life step (one lambda and eight nu per cell,
// Section "Exploring Compact Fractal Space").
#include "common.h"

namespace sqz {

namespace {

constexpr int kBlock = 256;

// Grid for a grid-stride loop over `count` items: enough workgroups to fill
// the device several times over, capped so 64-bit counters stay cheap.
inline unsigned grid_for(uint64_t count)
{
    uint64_t g = (count + kBlock - 1) / kBlock;
    if (g > 16384) g = 16384;
    if (g == 0) g = 1;
    return (unsigned)g;
}

__device__ __forceinline__ void lam_any(const MapParams &P, uint64_t c, uint32_t &x, uint32_t &y)
{
    if (P.N <= 0x100000000ull)
        lam_map32(P, (uint32_t)c, x, y);
    else
        lam_map64(P, c, x, y);
}

// The standalone maps stream their inputs from HBM: each lane takes kMapUnroll
// elements (kBlock apart, so every load instruction stays coalesced) per pass
// and issues all their loads before the first map, so the memory latency is
// paid once per kMapUnroll elements instead of once per element.
#ifndef SQZ_MAP_UNROLL
#define SQZ_MAP_UNROLL 8
#endif
constexpr int kMapUnroll = SQZ_MAP_UNROLL;

__global__ void __launch_bounds__(kBlock) k_lambda(MapParams P, const uint64_t *__restrict__ idx, int64_t count,
                                                   int32_t *__restrict__ xy)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock * kMapUnroll;
    for (int64_t i0 = (int64_t)blockIdx.x * kBlock * kMapUnroll + threadIdx.x; i0 < count; i0 += stride) {
        uint64_t c[kMapUnroll];
#pragma unroll
        for (int u = 0; u < kMapUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            c[u] = i < count ? idx[i] : ~0ull;
        }
#pragma unroll
        for (int u = 0; u < kMapUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            if (i < count) {
                int2 out = make_int2(-1, -1);
                if (c[u] < P.N) {
                    uint32_t x, y;
                    lam_any(P, c[u], x, y);
                    out = make_int2((int)x, (int)y);
                }
                reinterpret_cast<int2 *>(xy)[i] = out;
            }
        }
    }
}

// nu reads three table entries per point; each workgroup first copies the two
// nu tables into LDS (at most 2 x 4096 words) and then strides over the points.
__global__ void __launch_bounds__(kBlock) k_nu(MapParams P, const int32_t *__restrict__ xy, int64_t count,
                                               uint64_t *__restrict__ idx)
{
    extern __shared__ uint32_t s_nu[];
    const uint32_t nwords = P.ntab - (uint32_t)(P.nu_lo - P.lam_lo);
    for (uint32_t i = threadIdx.x; i < nwords; i += kBlock) s_nu[i] = P.nu_lo[i];
    __syncthreads();
    MapParams L = P;
    L.nu_lo = s_nu;
    L.nu_top = s_nu + (P.nu_top - P.nu_lo);
    const int64_t stride = (int64_t)gridDim.x * kBlock * kMapUnroll;
    for (int64_t i0 = (int64_t)blockIdx.x * kBlock * kMapUnroll + threadIdx.x; i0 < count; i0 += stride) {
        int2 p[kMapUnroll];
#pragma unroll
        for (int u = 0; u < kMapUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            p[u] = i < count ? reinterpret_cast<const int2 *>(xy)[i] : make_int2(0, 0);
        }
#pragma unroll
        for (int u = 0; u < kMapUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            if (i < count) idx[i] = nu_map(L, p[u].x, p[u].y);
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_fill_compact(MapParams P, uint64_t seed, uint32_t thresh,
                                                         uint8_t *__restrict__ out)
{
    for (uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x; c < P.N; c += (uint64_t)gridDim.x * kBlock) {
        uint32_t x, y;
        lam_any(P, c, x, y);
        uint64_t h = splitmix64_at(seed, (uint64_t)y * (uint64_t)P.n + x);
        out[c] = (uint8_t)((uint32_t)(h >> 40) < thresh);
    }
}

__global__ void __launch_bounds__(kBlock) k_fill_expanded(MapParams P, uint64_t seed, uint32_t thresh,
                                                          uint8_t *__restrict__ out)
{
    const uint64_t total = (uint64_t)P.n * (uint64_t)P.n;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (uint64_t)gridDim.x * kBlock) {
        uint32_t y = (uint32_t)(i / (uint32_t)P.n), x = (uint32_t)(i - (uint64_t)y * P.n);
        uint8_t v = 0;
        if (nu_map(P, (int32_t)x, (int32_t)y) != kHole64) v = (uint8_t)((uint32_t)(splitmix64_at(seed, i) >> 40) < thresh);
        out[i] = v;
    }
}

__global__ void __launch_bounds__(kBlock) k_fill_uniform(MapParams P, uint64_t seed, float *__restrict__ out)
{
    for (uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x; c < P.N; c += (uint64_t)gridDim.x * kBlock) {
        uint32_t x, y;
        lam_any(P, c, x, y);
        uint64_t h = splitmix64_at(seed, (uint64_t)y * (uint64_t)P.n + x);
        out[c] = (float)(uint32_t)(h >> 40) * (1.0f / 16777216.0f);
    }
}

// B3/S23 on the fractal: a member neighbour counts its state; a hole or a
// point outside the box counts nothing.
// One lambda and eight nu per cell make about 27 map-table reads per cell,
// scattered over tables of at most 4 x 4096 words.  Each workgroup copies
// the tables into LDS once and then strides over the cells, so those reads
// are LDS reads rather than divergent vector-memory gathers; only the nine
// state bytes per cell come through the vector-memory path.
constexpr int kCellBlock = 512;

__global__ void __launch_bounds__(kCellBlock) k_life_cell(MapParams P, const uint8_t *__restrict__ in,
                                                          uint8_t *__restrict__ out)
{
    extern __shared__ uint32_t s_tab[];
    for (uint32_t i = threadIdx.x; i < P.ntab; i += kCellBlock) s_tab[i] = P.lam_lo[i];
    __syncthreads();
    MapParams L = P;
    L.lam_lo = s_tab;
    L.lam_top = s_tab + (P.lam_top - P.lam_lo);
    L.nu_lo = s_tab + (P.nu_lo - P.lam_lo);
    L.nu_top = s_tab + (P.nu_top - P.lam_lo);
    for (uint64_t c = (uint64_t)blockIdx.x * kCellBlock + threadIdx.x; c < P.N;
         c += (uint64_t)gridDim.x * kCellBlock) {
        uint32_t x, y;
        lam_any(L, c, x, y);
        uint32_t cnt = 0;
        if (P.nnu >= 2) {
            // A neighbour inside the centre's lowest nu chunk shares every
            // higher chunk with it, so its index is the centre's with the
            // lowest chunk's digits replaced (nu(lambda(c)) = c): one table
            // read instead of a full nu.  Neighbours across the chunk edge
            // take the full map.
            const uint32_t hx = divq(x, P.dsnu), hy = divq(y, P.dsnu);
            const uint32_t lx = x - hx * P.snu, ly = y - hy * P.snu;
            const uint64_t chi = c - L.nu_lo[lx + P.snu * ly];
#pragma unroll
            for (int j = 0; j < 9; ++j) {
                if (j == 4) continue;
                const int dx = j % 3 - 1, dy = j / 3 - 1;
                const uint32_t nx = lx + (uint32_t)dx, ny = ly + (uint32_t)dy;
                uint64_t q;
                if (nx < P.snu && ny < P.snu) {
                    const uint32_t e = L.nu_lo[nx + P.snu * ny];
                    q = e == kNuHole32 ? kHole64 : chi + e;
                } else {
                    q = nu_map(L, (int32_t)x + dx, (int32_t)y + dy);
                }
                if (q != kHole64) cnt += in[q];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 9; ++j) {
                if (j == 4) continue;
                int dx = j % 3 - 1, dy = j / 3 - 1;
                uint64_t q = nu_map(L, (int32_t)x + dx, (int32_t)y + dy);
                if (q != kHole64) cnt += in[q];
            }
        }
        uint32_t self = in[c];
        out[c] = (uint8_t)(cnt == 3 || (self && cnt == 2));
    }
}

sqz_status after_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, what);
}

}  // namespace

sqz_status launch_lambda(const MapParams &P, const uint64_t *idx, int64_t count, int32_t *xy, hipStream_t st)
{
    hipLaunchKernelGGL(k_lambda, dim3(grid_for((uint64_t)count)), dim3(kBlock), 0, st, P, idx, count, xy);
    return after_launch("lambda_map launch");
}

sqz_status launch_nu(const MapParams &P, const int32_t *xy, int64_t count, uint64_t *idx, hipStream_t st)
{
    // as many workgroups as are resident at once (each copies the tables once),
    // and no more than the points need
    const size_t lds = (size_t)(P.ntab - (uint32_t)(P.nu_lo - P.lam_lo)) * sizeof(uint32_t);
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_nu, kBlock, lds);
    if (e != hipSuccess) return hip_error(e, "nu_map occupancy");
    if (per_cu < 1) return set_error(SQZ_ERR_UNSUPPORTED, "nu tables (%zu B) do not fit in LDS", lds);
    uint64_t grid = ((uint64_t)count + (uint64_t)kBlock * kMapUnroll - 1) / ((uint64_t)kBlock * kMapUnroll);
    if (grid > (uint64_t)cus * per_cu) grid = (uint64_t)cus * per_cu;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(k_nu, dim3((unsigned)grid), dim3(kBlock), lds, st, P, xy, count, idx);
    return after_launch("nu_map launch");
}

sqz_status launch_fill_bernoulli(const MapParams &P, uint64_t seed, uint32_t thresh24, int expanded, uint8_t *out,
                                 hipStream_t st)
{
    if (expanded) {
        uint64_t total = (uint64_t)P.n * (uint64_t)P.n;
        hipLaunchKernelGGL(k_fill_expanded, dim3(grid_for(total)), dim3(kBlock), 0, st, P, seed, thresh24, out);
    } else {
        hipLaunchKernelGGL(k_fill_compact, dim3(grid_for(P.N)), dim3(kBlock), 0, st, P, seed, thresh24, out);
    }
    return after_launch("fill_bernoulli launch");
}

sqz_status launch_fill_uniform(const MapParams &P, uint64_t seed, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_uniform, dim3(grid_for(P.N)), dim3(kBlock), 0, st, P, seed, out);
    return after_launch("fill_uniform launch");
}

sqz_status launch_life_cell(const MapParams &P, const uint8_t *in, uint8_t *out, hipStream_t st)
{
    // as many workgroups as are resident at once: each copies the tables once
    const size_t lds = (size_t)P.ntab * sizeof(uint32_t);
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_life_cell, kCellBlock, lds);
    if (e != hipSuccess) return hip_error(e, "compact_step (cell) occupancy");
    if (per_cu < 1) return set_error(SQZ_ERR_UNSUPPORTED, "map tables (%zu B) do not fit in LDS", lds);
    uint64_t grid = (P.N + kCellBlock - 1) / kCellBlock;
    if (grid > (uint64_t)cus * per_cu) grid = (uint64_t)cus * per_cu;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(k_life_cell, dim3((unsigned)grid), dim3(kCellBlock), lds, st, P, in, out);
    return after_launch("compact_step (cell) launch");
}

}  // namespace sqz
