// Bit-sliced block-level Life kernels (device code in tile_device.h) and
// their host-side preparation: tile halo slots, block-halo tables, per-tile
// halo indices.
#include <type_traits>
#include <vector>

#include "tile_device.h"

namespace sqz {

#ifndef SQZ_TILE_NT  // lanes per workgroup of the compact tiled kernels
#define SQZ_TILE_NT 256
#endif
constexpr int kTileNT = SQZ_TILE_NT;

// Lanes per workgroup of a pattern's tiled kernels: 512 for the level-10
// tiles of large triangles (2,187 blocks), else kTileNT.
template <class Pat>
constexpr int nt_of()
{
    return std::is_same<Pat, PatTriangleBig>::value ? 512 : kTileNT;
}

template <class Pat, int NT>
__global__ void __launch_bounds__(NT) k_life_tile(TileArgs A, const uint8_t *__restrict__ in,
                                                  uint8_t *__restrict__ out)
{
    using LDS = TileLds<Pat>;
    __shared__ uint32_t s_in[LDS::WORDS];
    __shared__ uint32_t s_out[LDS::WORDS];
    const uint32_t G = gridDim.x;
    for (uint64_t round = 0; round * G < A.ntiles; ++round) {
        const uint64_t t = round * G + xcd_remap(blockIdx.x, G);
        if (t >= A.ntiles) break;  // uniform across the workgroup
        tile_body<Pat, NT>(A, in, out, t, s_in, s_out);
    }
}

template <class Pat, int K, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 256 ? 8 : 7)))
k_life_tileK(TileArgs A, const uint8_t *__restrict__ in, uint8_t *__restrict__ out)
{
    using LDS = TileLds<Pat>;
    __shared__ uint32_t s_buf[3][LDS::WORDS];
    __shared__ __align__(16) uint32_t s_ring[kRingTab];
    uint32_t *const buf[3] = {s_buf[0], s_buf[1], s_buf[2]};
    const uint32_t G = gridDim.x;
    for (uint64_t round = 0; round * G < A.ntiles; ++round) {
        const uint64_t t = round * G + xcd_remap(blockIdx.x, G);
        if (t >= A.ntiles) break;  // uniform across the workgroup
        tile_bodyK<Pat, K, NT>(A, in, out, t, buf, s_ring);
    }
}

// Tile-halo cells of every tile: global compact index of each slot's cell.
__global__ void __launch_bounds__(kBlock) k_tile_halo(MapParams Pc, uint64_t ntiles, uint32_t nthalo,
                                                      uint64_t tile_cells, const int4 *__restrict__ slots,
                                                      uint64_t *__restrict__ outp)
{
    for (uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x; t < ntiles; t += (uint64_t)gridDim.x * kBlock) {
        uint32_t X, Y;
        if (Pc.N <= 0x100000000ull)
            lam_map32(Pc, (uint32_t)t, X, Y);
        else
            lam_map64(Pc, t, X, Y);
        for (uint32_t j = 0; j < nthalo; ++j) {
            const int4 sl = slots[j];  // (tile dx, tile dy, cell index in that tile, unused)
            const uint64_t nt = nu_map(Pc, (int32_t)X + sl.x, (int32_t)Y + sl.y);
            outp[t * nthalo + j] = nt == kHole64 ? kHole64 : nt * tile_cells + (uint64_t)sl.z;
        }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {

template <class Pat>
bool matches(const FractalHost &F)
{
    if (F.s != Pat::S || F.k != Pat::K) return false;
    for (int j = 0; j < Pat::K; ++j)
        if (F.ox[j] != Pat::OX[j] || F.oy[j] != Pat::OY[j]) return false;
    return true;
}

template <class Pat>
sqz_status prepare(FractalHost &F)
{
    constexpr const BlockPlan &PL = PlanOf<Pat>::value;
    constexpr int J = Pat::J;
    TileConfig *T = new TileConfig();
    const int mtop = F.r >= Pat::MBIG ? Pat::MMAX : (Pat::MSMALL < Pat::MMAX ? Pat::MSMALL : Pat::MMAX);
    T->M = F.r < mtop ? F.r : mtop;
    const int M = T->M;
    T->tile = (uint32_t)cpow(Pat::K, M);
    T->nblocks = (uint32_t)cpow(Pat::K, M - J);
    using LDS = TileLds<Pat>;
    const int64_t side = cpow(Pat::S, M), box = PL.box;

    // tile halo slots: cells of adjacent tiles that touch a cell of this tile
    struct Slot {
        int dx, dy;
        int64_t idx, px, py;  // cell index in the neighbour tile; position relative to this tile
    };
    std::vector<Slot> slots;
    for (uint64_t c = 0; c < T->tile; ++c) {
        int64_t x, y;
        host_lambda(F, M, c, x, y);
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int64_t qx = x + dx, qy = y + dy;
                if (qx >= 0 && qy >= 0 && qx < side && qy < side) continue;
                const int tdx = qx < 0 ? -1 : (qx >= side ? 1 : 0), tdy = qy < 0 ? -1 : (qy >= side ? 1 : 0);
                const int64_t j = host_nu(F, M, qx - tdx * side, qy - tdy * side);
                if (j < 0) continue;
                bool seen = false;
                for (const Slot &s : slots) seen |= s.px == qx && s.py == qy;
                if (!seen) slots.push_back(Slot{tdx, tdy, j, qx, qy});
            }
    }
    if (slots.size() > (size_t)kMaxTileHalo) {
        delete T;
        return set_error(SQZ_ERR_UNSUPPORTED, "tile halo of %zu cells exceeds %d", slots.size(), kMaxTileHalo);
    }
    T->nthalo = (uint32_t)slots.size();

    // rings 2..kMaxSteps (several steps per launch): breadth-first from ring 1
    // over member cells outside the tile (ring d = graph distance d from the
    // tile); all rings must fit kMaxRing lanes.
    std::vector<Slot> ring = slots;  // rings in order, ring 1 first
    std::vector<uint32_t> start = {0, (uint32_t)slots.size()};
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
    uint32_t ksteps = 1;
    for (int d = 2; d <= kMaxSteps; ++d) {
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
        // (ring cells must also lie in adjacent tiles: d < side)
        if (T->nthalo == 0 || start[d] > (uint32_t)kMaxRing || d >= side) break;
        ksteps = (uint32_t)d;  // rings 1..d fit: d steps per launch
    }
    T->ksteps = ksteps;
    for (int d = 0; d <= kMaxSteps; ++d) T->ring_start[d] = start[d <= (int)ksteps ? d : ksteps];
    T->tstride = T->ring_start[ksteps];
    T->nsrc = ksteps >= 2 ? T->ring_start[ksteps - 1] : 0;
    ring.resize(T->tstride);

    // adjacent blocks of other tiles that hold ring-1 cells (one LDS word each)
    auto floor_div = [](int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
    std::vector<std::pair<int64_t, int64_t>> vblk;
    auto virt_of = [&](int64_t bx, int64_t by) {
        for (size_t g = 0; g < vblk.size(); ++g)
            if (vblk[g].first == bx && vblk[g].second == by) return (int64_t)g;
        return (int64_t)-1;
    };
    for (const Slot &s : slots) {
        const int64_t bx = floor_div(s.px, box), by = floor_div(s.py, box);
        if (virt_of(bx, by) < 0) vblk.emplace_back(bx, by);
    }
    // LDS entry (byte offset of the word << 16 | bit) of a tile cell and of ring cell i
    auto entry = [](uint32_t word, uint32_t bit) { return (4u * word) << 16 | bit; };
    const uint32_t zero_entry = entry(LDS::ZERO, 0);
    auto tile_entry = [&](int64_t j) { return entry((uint32_t)(j / PL.nc), (uint32_t)(j % PL.nc)); };
    auto ring_entry = [&](size_t i) {
        uint32_t d = 1;
        while ((uint32_t)i >= T->ring_start[d]) ++d;
        if (d == 1) {
            const Slot &s = ring[i];
            const int64_t g = virt_of(floor_div(s.px, box), floor_div(s.py, box));
            return entry(LDS::VIRT + (uint32_t)g, (uint32_t)(s.idx % PL.nc));
        }
        const uint32_t k = (uint32_t)i - T->nthalo;  // rings 2.. packed in order
        return entry(LDS::RING2 + k / 32, k % 32);
    };
    std::vector<uint32_t> home(T->tstride ? T->tstride : 1, zero_entry);
    for (uint32_t i = 0; i < T->tstride; ++i) home[i] = ring_entry(i);
    // LDS sources of the neighbours of every ring cell that is advanced
    std::vector<uint32_t> rsrc(T->nsrc ? (size_t)T->nsrc * 8 : 1, zero_entry);
    for (uint32_t c = 0; c < T->nsrc; ++c) {
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
                        if (i >= 0 && i < (int64_t)T->tstride) e = ring_entry((size_t)i);
                    }
                }
                rsrc[(size_t)c * 8 + n++] = e;
            }
    }

    // adjacent-block words of every block: a block of the tile, the word of
    // an adjacent block of another tile, or a zero word (no such block)
    const int NG = PL.ngrp, NP = (NG + 1) / 2;
    T->nbstride = NP > 4 ? (uint32_t)((NP + 3) / 4 * 4) : 4u;
    std::vector<uint32_t> nbt((size_t)T->nblocks * T->nbstride, 0);
    const int64_t bside = cpow(Pat::S, M - J);
    for (uint32_t b = 0; b < T->nblocks; ++b) {
        int64_t bx, by;
        host_lambda(F, M - J, b, bx, by);
        for (int g = 0; g < NG; ++g) {
            const int64_t nbx = bx + PL.g_dx[g], nby = by + PL.g_dy[g];
            uint32_t w = LDS::ZERO;
            if (nbx >= 0 && nby >= 0 && nbx < bside && nby < bside) {
                const int64_t nb = host_nu(F, M - J, nbx, nby);
                if (nb >= 0) w = (uint32_t)nb;
            } else {
                const int64_t v = virt_of(nbx, nby);
                if (v >= 0) w = LDS::VIRT + (uint32_t)v;
            }
            nbt[(size_t)b * T->nbstride + g / 2] |= (4u * w) << (16 * (g & 1));
        }
    }

    // coarse maps and per-tile halo indices
    sqz_status st = build_map_params(F, F.r - M, T->Pc, &T->d_coarse_tables);
    if (st != SQZ_OK) {
        delete T;
        return st;
    }
    T->ntiles = T->Pc.N;
    T->d_nbtab = nullptr;
    T->d_tile_halo = nullptr;
    T->d_ringsrc = nullptr;
    T->d_ringhome = nullptr;
    int4 *d_slots = nullptr;
    std::vector<int4> hs(T->tstride ? T->tstride : 1);
    for (size_t s = 0; s < T->tstride; ++s) hs[s] = make_int4(ring[s].dx, ring[s].dy, (int)ring[s].idx, 0);
    auto upload = [](uint32_t **d, const std::vector<uint32_t> &h) {
        hipError_t e = hipMalloc(d, h.size() * sizeof(uint32_t));
        return e == hipSuccess ? hipMemcpy(*d, h.data(), h.size() * sizeof(uint32_t), hipMemcpyHostToDevice) : e;
    };
    hipError_t e = upload(&T->d_nbtab, nbt);
    if (e == hipSuccess) e = upload(&T->d_ringsrc, rsrc);
    if (e == hipSuccess) e = upload(&T->d_ringhome, home);
    if (e == hipSuccess)
        e = hipMalloc(&T->d_tile_halo, (size_t)T->ntiles * (T->tstride ? T->tstride : 1) * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&d_slots, hs.size() * sizeof(int4));
    if (e == hipSuccess) e = hipMemcpy(d_slots, hs.data(), hs.size() * sizeof(int4), hipMemcpyHostToDevice);
    if (e == hipSuccess && T->tstride) {
        uint64_t g = (T->ntiles + kBlock - 1) / kBlock;
        if (g > 16384) g = 16384;
        hipLaunchKernelGGL(k_tile_halo, dim3((unsigned)g), dim3(kBlock), 0, 0, T->Pc, T->ntiles, T->tstride,
                           (uint64_t)T->tile, d_slots, T->d_tile_halo);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (d_slots) (void)hipFree(d_slots);
    if (e != hipSuccess) {
        if (T->d_nbtab) (void)hipFree(T->d_nbtab);
        if (T->d_tile_halo) (void)hipFree(T->d_tile_halo);
        if (T->d_ringsrc) (void)hipFree(T->d_ringsrc);
        if (T->d_ringhome) (void)hipFree(T->d_ringhome);
        (void)hipFree(T->d_coarse_tables);
        delete T;
        return hip_error(e, "tile table setup");
    }
    F.tile = T;
    return SQZ_OK;
}

template <class Pat>
sqz_status launch(const FractalHost &F, const uint8_t *in, uint8_t *out, int steps, hipStream_t st)
{
    const TileConfig *T = F.tile;
    if (((uintptr_t)in & 15) || ((uintptr_t)out & 15))
        return set_error(SQZ_ERR_INVALID, "tiled kernel needs 16-byte aligned buffers");
    if (steps < 1 || steps > (int)T->ksteps)
        return set_error(SQZ_ERR_UNSUPPORTED, "%d steps per launch exceed the %u this fractal's tiles allow", steps,
                         T->ksteps);
    const TileArgs A = tile_args(F);
    const uint64_t grid = T->ntiles < (1ull << 20) ? T->ntiles : (1ull << 20);
    constexpr int NT = nt_of<Pat>();
    switch (steps) {
    case 1: hipLaunchKernelGGL((k_life_tile<Pat, NT>), dim3((unsigned)grid), dim3(NT), 0, st, A, in, out); break;
    case 2: hipLaunchKernelGGL((k_life_tileK<Pat, 2, NT>), dim3((unsigned)grid), dim3(NT), 0, st, A, in, out); break;
    case 3: hipLaunchKernelGGL((k_life_tileK<Pat, 3, NT>), dim3((unsigned)grid), dim3(NT), 0, st, A, in, out); break;
    case 4: hipLaunchKernelGGL((k_life_tileK<Pat, 4, NT>), dim3((unsigned)grid), dim3(NT), 0, st, A, in, out); break;
    case 5: hipLaunchKernelGGL((k_life_tileK<Pat, 5, NT>), dim3((unsigned)grid), dim3(NT), 0, st, A, in, out); break;
    case 6: hipLaunchKernelGGL((k_life_tileK<Pat, 6, NT>), dim3((unsigned)grid), dim3(NT), 0, st, A, in, out); break;
    case 7: hipLaunchKernelGGL((k_life_tileK<Pat, 7, NT>), dim3((unsigned)grid), dim3(NT), 0, st, A, in, out); break;
    case 8: hipLaunchKernelGGL((k_life_tileK<Pat, 8, NT>), dim3((unsigned)grid), dim3(NT), 0, st, A, in, out); break;
    case 9: hipLaunchKernelGGL((k_life_tileK<Pat, 9, NT>), dim3((unsigned)grid), dim3(NT), 0, st, A, in, out); break;
    default: hipLaunchKernelGGL((k_life_tileK<Pat, 10, NT>), dim3((unsigned)grid), dim3(NT), 0, st, A, in, out); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "compact step (tile) launch");
}

enum { kNone = 0, kTriangle = 1, kTrianglePaper = 2, kVicsek = 3, kTriangleBig = 4 };

}  // namespace

int tile_kind_for(const FractalHost &F)
{
    if (matches<PatTriangle>(F) && F.r >= SQZ_TRI_TILE_BIG_FROM) return kTriangleBig;
    if (matches<PatTriangle>(F) && F.r >= PatTriangle::J) return kTriangle;
    if (matches<PatTrianglePaper>(F) && F.r >= PatTrianglePaper::J) return kTrianglePaper;
    if (matches<PatVicsek>(F) && F.r >= PatVicsek::J) return kVicsek;
    return kNone;
}

sqz_status tile_prepare(FractalHost &F)
{
    switch (F.tile_kind) {
    case kTriangle: return prepare<PatTriangle>(F);
    case kTriangleBig: return prepare<PatTriangleBig>(F);
    case kTrianglePaper: return prepare<PatTrianglePaper>(F);
    case kVicsek: return prepare<PatVicsek>(F);
    }
    return set_error(SQZ_ERR_UNSUPPORTED, "no tiled kernel");
}

void tile_release(FractalHost &F)
{
    if (!F.tile) return;
    (void)hipFree(F.tile->d_nbtab);
    (void)hipFree(F.tile->d_tile_halo);
    (void)hipFree(F.tile->d_ringsrc);
    (void)hipFree(F.tile->d_ringhome);
    (void)hipFree(F.tile->d_coarse_tables);
    delete F.tile;
    F.tile = nullptr;
}

int32_t tile_level_of(const FractalHost &F) { return F.tile ? F.tile->M : 0; }

sqz_status launch_life_tile(const FractalHost &F, const uint8_t *in, uint8_t *out, hipStream_t st)
{
    return launch_life_tile_steps(F, in, out, 1, st);
}

int tile_steps_per_launch(const FractalHost &F) { return F.tile ? (int)F.tile->ksteps : 0; }

sqz_status launch_life_tile_steps(const FractalHost &F, const uint8_t *in, uint8_t *out, int steps, hipStream_t st)
{
    switch (F.tile_kind) {
    case kTriangle: return launch<PatTriangle>(F, in, out, steps, st);
    case kTriangleBig: return launch<PatTriangleBig>(F, in, out, steps, st);
    case kTrianglePaper: return launch<PatTrianglePaper>(F, in, out, steps, st);
    case kVicsek: return launch<PatVicsek>(F, in, out, steps, st);
    }
    return set_error(SQZ_ERR_UNSUPPORTED, "no tiled kernel");
}

}  // namespace sqz
