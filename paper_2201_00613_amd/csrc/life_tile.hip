// Bit-sliced block-level Life kernels (device code in tile_device.h) and
// their host-side preparation: tile halo slots, block-halo tables, per-tile
// halo indices.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "tile_device.h"

namespace sqz {

#ifndef SQZ_TILE_NT  // lanes per workgroup of the compact tiled kernels
#define SQZ_TILE_NT 256
#endif
constexpr int kTileNT = SQZ_TILE_NT;

#ifndef SQZ_BIG_NT  // lanes per workgroup of the level-10 triangle tiles
#define SQZ_BIG_NT 512
#endif
#ifndef SQZ_TILEK_FULL  // 1: the multi-step launches run whole slots without a branch (more registers)
#define SQZ_TILEK_FULL 0
#endif
#ifndef SQZ_BIG_WAVES  // minimum waves per SIMD (register budget) of their multi-step kernels
#define SQZ_BIG_WAVES 7
#endif

// Lanes per workgroup of a pattern's tiled kernels: SQZ_BIG_NT for the
// level-10 tiles of large triangles (2,187 blocks), else kTileNT.
template <class Pat>
constexpr int nt_of()
{
    return std::is_same<Pat, PatTriangleBig>::value ? SQZ_BIG_NT : kTileNT;
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
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 256 ? 8 : SQZ_BIG_WAVES)))
k_life_tileK(TileArgs A, const uint8_t *__restrict__ in, uint8_t *__restrict__ out)
{
    using LDS = TileLds<Pat>;
    __shared__ uint32_t s_buf[3][LDS::WORDS];
    __shared__ __align__(16) uint32_t s_ring[kRingTab];
    uint32_t *const buf[3] = {s_buf[0], s_buf[1], s_buf[2]};
    const uint32_t G = gridDim.x;
    const bool full = SQZ_TILEK_FULL && A.nblocks == LDS::NBMAX;  // every tile has the pattern's largest level
    for (uint64_t round = 0; round * G < A.ntiles; ++round) {
        const uint64_t t = round * G + xcd_remap(blockIdx.x, G);
        if (t >= A.ntiles) break;  // uniform across the workgroup
        if (full)
            tile_bodyK<Pat, K, NT, true>(A, in, out, t, buf, s_ring);
        else
            tile_bodyK<Pat, K, NT>(A, in, out, t, buf, s_ring);
    }
}

#ifndef SQZ_RESIDENT_PAD  // LDS reserved per workgroup of the resident run (bytes; balance, see prepare_resident)
#define SQZ_RESIDENT_PAD(pad) (pad)
#endif

// Resident run: one workgroup per tile for all steps, every tile on the chip at once
// (at most ceil(tiles / CUs) workgroups per CU: six waves per SIMD for the level-16
// triangle, so the register budget is that of six).
template <class Pat, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 256 ? 8 : (SQZ_RES_STATIC ? 6 : SQZ_BIG_WAVES))))
k_life_tileR(TileArgs A, ResidentArgs P)
{
    using LDS = TileLds<Pat>;
    __shared__ uint32_t s_buf[3 * LDS::WORDS];
    __shared__ __align__(16) uint32_t s_ring[kRingTab];
    __shared__ uint32_t s_rs[kMaxSteps + 1];
    tile_bodyR<Pat, NT>(A, P, xcd_remap(blockIdx.x, gridDim.x), s_buf, s_ring, s_rs);
}

__global__ void k_zero_words(uint32_t *p, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
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

// The resident run is offered when every tile fits on the chip at once (one
// workgroup per tile, occupancy from the kernel's registers and LDS) and the
// tiles take at least two steps between exchanges.  Failure to set it up only
// leaves it unavailable.
template <class Pat>
void prepare_resident(FractalHost &F, const TileTables &TT)
{
    TileConfig *T = F.tile;
    constexpr int NT = nt_of<Pat>();
    if (T->ksteps < 2 || TT.bound.empty()) return;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_life_tileR<Pat, NT>, NT, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, F.device) != hipSuccess || cus < 1)
        return;
    // The occupancy query counts waves per CU, but a workgroup's waves are dealt
    // to the CU's four SIMDs, so one of them takes ceil(waves / 4): with the
    // per-SIMD wave limit of the kernel's registers, that bounds the workgroups a
    // CU holds at once.  A grid larger than what surely fits is never resident.
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_life_tileR<Pat, NT>)) != hipSuccess) return;
    {
        const int vgprs = fa.numRegs > 0 ? (fa.numRegs + 7) / 8 * 8 : 512;
        const int simd_waves = std::min(8, 512 / vgprs), wg_simd = (NT / 64 + 3) / 4;
        per_cu = std::min(per_cu, simd_waves / wg_simd);
    }
    if ((uint64_t)per_cu * (uint64_t)cus < T->ntiles) return;
    // Balance: a CU that receives more tiles than ceil(tiles / CUs) sets the time of
    // every round, so reserve unused LDS per workgroup until no more than that many
    // fit on a CU (the smallest such reservation, found with the occupancy query).
    const int target = (int)((T->ntiles + (uint64_t)cus - 1) / (uint64_t)cus);
    uint32_t pad = 0;
    int lds_cu = 0;
    if (per_cu > target &&
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, F.device) == hipSuccess &&
        (size_t)lds_cu / (size_t)target > fa.sharedSizeBytes) {
        // occupancy(lo) > target; find the least hi with occupancy <= target
        uint32_t lo = 0, hi = (uint32_t)((size_t)lds_cu / (size_t)target - fa.sharedSizeBytes);
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_life_tileR<Pat, NT>, NT, hi) == hipSuccess &&
            occ <= target && occ >= 1) {
            while (hi - lo > 256) {
                const uint32_t mid = (lo + hi) / 2;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_life_tileR<Pat, NT>, NT, mid) != hipSuccess)
                    break;
                (occ <= target ? hi : lo) = mid;
            }
            int lds_wg = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_life_tileR<Pat, NT>, NT, hi) == hipSuccess &&
                occ == target &&
                hipDeviceGetAttribute(&lds_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, F.device) == hipSuccess &&
                fa.sharedSizeBytes + hi <= (size_t)lds_wg)
                pad = hi;
        }
        (void)hipGetLastError();
    }
    T->lds_pad = pad;
    uint32_t *d_bound = nullptr, *d_bar = nullptr, *h_flag = nullptr;
    hipError_t e = hipMalloc(&d_bound, TT.bound.size() * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMemcpy(d_bound, TT.bound.data(), TT.bound.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&d_bar, bar_words(T->ntiles) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(d_bar, 0, bar_words(T->ntiles) * sizeof(uint32_t));  // counts carry over between runs
    if (e == hipSuccess) e = hipHostMalloc(&h_flag, sizeof(uint32_t), hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (d_bound) (void)hipFree(d_bound);
        if (d_bar) (void)hipFree(d_bar);
        return;
    }
    *h_flag = 0;
    T->nbound = (uint32_t)TT.bound.size();
    T->d_bound = d_bound;
    T->d_bar = d_bar;
    T->h_flag = h_flag;
}

template <class Pat>
sqz_status launch_resident(const FractalHost &F, uint8_t *a, uint8_t *b, int steps, hipStream_t st)
{
    const TileConfig *T = F.tile;
    if (__atomic_exchange_n(T->h_flag, 0u, __ATOMIC_ACQ_REL)) {
        // the counts of the failed run are unknown: clear them for the next run
        hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, st, T->d_bar, bar_words(T->ntiles));
        (void)hipGetLastError();
        return set_error(SQZ_ERR_HIP, "a grid barrier of an earlier resident run timed out: its result is invalid");
    }
    constexpr int NT = nt_of<Pat>();
    TileArgs A = tile_args(F);
    ResidentArgs P;
    P.a = a;
    P.b = b;
    P.steps = steps;
    P.kstep = (int32_t)T->ksteps;
    P.nbound = T->nbound;
    P.bound = T->d_bound;
    P.bar = T->d_bar;
    P.flag = T->h_flag;
    // An ordinary launch: the occupancy check at set-up guarantees that the grid
    // fits the chip at once, so on an otherwise idle device every workgroup is
    // resident; a workgroup that waits for the chip to be shared with other work
    // starts when that work ends, and the bounded barrier wait catches the rest.
    hipLaunchKernelGGL((k_life_tileR<Pat, NT>), dim3((unsigned)T->ntiles), dim3(NT), SQZ_RESIDENT_PAD(T->lds_pad), st,
                       A, P);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "resident run launch");
}

template <class Pat>
sqz_status prepare(FractalHost &F)
{
    constexpr const BlockPlan &PL = PlanOf<Pat>::value;
    using LDS = TileLds<Pat>;
    TileConfig *T = new TileConfig();
    const int mtop = F.r >= Pat::MBIG ? Pat::MMAX : (Pat::MSMALL < Pat::MMAX ? Pat::MSMALL : Pat::MMAX);
    T->M = F.r < mtop ? F.r : mtop;
    const int M = T->M;
    T->tile = (uint32_t)cpow(Pat::K, M);
    T->nblocks = (uint32_t)cpow(Pat::K, M - Pat::J);

    // tables of the tile (the same for every tile): rings, halos, LDS entries
    TileSpec S;
    S.M = M;
    S.J = Pat::J;
    S.nc = PL.nc;
    S.box = PL.box;
    S.ngrp = PL.ngrp;
    for (int g = 0; g < 8; ++g) {
        S.g_dx[g] = g < PL.ngrp ? PL.g_dx[g] : 0;
        S.g_dy[g] = g < PL.ngrp ? PL.g_dy[g] : 0;
    }
    S.lds_zero = LDS::ZERO;
    S.lds_virt = LDS::VIRT;
    S.lds_ring2 = LDS::RING2;
    S.max_tile_halo = kMaxTileHalo;
    S.max_ring = kMaxRing;
    S.max_steps = kMaxSteps;
    TileTables TT;
    if (tile_tables(F, S, TT) != SQZ_OK) {
        delete T;
        return SQZ_ERR_UNSUPPORTED;
    }
    T->nthalo = TT.nthalo;
    T->ksteps = TT.ksteps;
    for (int d = 0; d <= kMaxSteps; ++d) T->ring_start[d] = TT.ring_start[d];
    T->tstride = TT.tstride;
    T->nsrc = TT.nsrc;
    T->nbstride = TT.nbstride;
    const std::vector<uint32_t> &nbt = TT.nbt, &rsrc = TT.rsrc, &home = TT.home;

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
    std::vector<int4> hs(T->tstride ? T->tstride : 1, make_int4(0, 0, 0, 0));
    for (size_t s = 0; s < T->tstride; ++s)
        hs[s] = make_int4(TT.slots[4 * s], TT.slots[4 * s + 1], TT.slots[4 * s + 2], 0);
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
    T->nbound = 0;
    T->lds_pad = 0;
    T->d_bound = nullptr;
    T->d_bar = nullptr;
    T->h_flag = nullptr;
    F.tile = T;
    prepare_resident<Pat>(F, TT);
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
    if (F.tile->d_bound) (void)hipFree(F.tile->d_bound);
    if (F.tile->d_bar) (void)hipFree(F.tile->d_bar);
    if (F.tile->h_flag) (void)hipHostFree(F.tile->h_flag);
    delete F.tile;
    F.tile = nullptr;
}

int32_t tile_level_of(const FractalHost &F) { return F.tile ? F.tile->M : 0; }

sqz_status launch_life_tile(const FractalHost &F, const uint8_t *in, uint8_t *out, hipStream_t st)
{
    return launch_life_tile_steps(F, in, out, 1, st);
}

int tile_steps_per_launch(const FractalHost &F) { return F.tile ? (int)F.tile->ksteps : 0; }

bool tile_resident(const FractalHost &F) { return F.tile && F.tile->d_bar; }

sqz_status launch_life_tile_resident(const FractalHost &F, uint8_t *a, uint8_t *b, int steps, hipStream_t st)
{
    if (!tile_resident(F)) return set_error(SQZ_ERR_UNSUPPORTED, "the tiles of this fractal do not fit the chip at once");
    if (((uintptr_t)a & 15) || ((uintptr_t)b & 15))
        return set_error(SQZ_ERR_INVALID, "tiled kernel needs 16-byte aligned buffers");
    if (steps < 1) return SQZ_OK;
    switch (F.tile_kind) {
    case kTriangle: return launch_resident<PatTriangle>(F, a, b, steps, st);
    case kTriangleBig: return launch_resident<PatTriangleBig>(F, a, b, steps, st);
    case kTrianglePaper: return launch_resident<PatTrianglePaper>(F, a, b, steps, st);
    case kVicsek: return launch_resident<PatVicsek>(F, a, b, steps, st);
    }
    return set_error(SQZ_ERR_UNSUPPORTED, "no tiled kernel");
}

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
