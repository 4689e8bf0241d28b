// Batched Life: many independent fractals of mixed replica pattern and level
// advanced together.
//
// Every instance owns a 256-byte aligned range of one state buffer.
// Instances with a tiled kernel (bit-sliced tiles of the triangle, its mirror
// image and the Vicsek cross; bit rows of the carpet) run in one of two
// forms: one launch per pattern group, with one workgroup per tile of any of
// the group's instances and the group's own steps per launch; or one
// persistent launch over all of them, in which workgroup b takes the tiles
// whose first cell falls in the b-th equal share of their cells.  The tile
// bodies are the single-fractal kernels' device functions.  The remaining
// instances (expanded tiles of any pattern, runs of 4096 cells of the
// thread-level path for instances too small to tile) share one persistent
// launch balanced the same way by a per-path cost; the expanded-tile tables
// are reloaded only when a workgroup moves to an instance with a different
// tile configuration.  Instances are independent, so every launch form
// follows its own plan of launches; each plan has the parity of the step
// count, so all results land in the same buffer.
//
// Runs of several steps are captured once into a hipGraph (kernel nodes only)
// and replayed; an autotuner times the launch forms, steps per launch and
// grid sizes on the caller's buffers and keeps the fastest, cached per batch
// composition.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bitbox_device.h"
#include "tile_device.h"
#include "xtile_device.h"

struct sqz_fractal;  // api.hip

namespace sqz {

enum BatchKind : uint32_t { kBTri = 1, kBTriPaper = 2, kBVicsek = 3, kBX68 = 4, kBX84 = 5, kBXAny = 6, kBCell = 7, kBBits = 8 };
#ifndef SQZ_BATCH_TILE_MAP  // 1: the workgroup-per-tile launch interleaves the kinds tile by tile
#define SQZ_BATCH_TILE_MAP 1
#endif
#ifndef SQZ_BATCH_INTERLEAVE  // 1: tiled launches take the pattern kinds evenly interleaved
#define SQZ_BATCH_INTERLEAVE 1
#endif

constexpr uint32_t kCellUnit = 4096;

struct BatchInst {
    uint32_t kind, xcfg;   // xcfg: expanded-tile configuration id (LDS tables)
    uint64_t base;         // byte offset of the instance in the state buffer
    uint64_t units;        // work units
    uint64_t unit_cells;   // cells per unit
    uint64_t cell_start;   // first cell of the instance in the batch's cell sequence
    uint64_t cost_start;   // first cost unit of the instance (cells weighted by path)
    uint64_t unit_cost;    // cost of one work unit
    uint64_t cells;
    TileArgs tile;
    XArgs x;
    XArgs xk;  // multi-step expanded tiles (LDS offsets of the Life layout)
    MapParams P;
};

struct BatchArgs {
    const BatchInst *inst;
    const uint64_t *cost_start;  // ninst + 1 entries
    uint32_t ninst;
    uint64_t total_cost;
};

namespace {

__device__ __forceinline__ void life_cell_unit(const MapParams &P, const uint8_t *in, uint8_t *out, uint64_t unit)
{
    const uint64_t c0 = unit * kCellUnit;
    for (uint32_t k = threadIdx.x; k < kCellUnit; k += 256) {
        const uint64_t c = c0 + k;
        if (c >= P.N) break;
        uint32_t x, y;
        if (P.N <= 0x100000000ull)
            lam_map32(P, (uint32_t)c, x, y);
        else
            lam_map64(P, c, x, y);
        uint32_t cnt = 0;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            if (j == 4) continue;
            const uint64_t q = nu_map(P, (int32_t)x + j % 3 - 1, (int32_t)y + j / 3 - 1);
            if (q != kHole64) cnt += in[q];
        }
        const uint32_t self = in[c];
        out[c] = (uint8_t)(cnt == 3 || (self && cnt == 2));
    }
}

// K Life steps of every instance of the persistent launch (K > 1: every such
// instance has multi-step expanded tiles).
template <int K>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_batch_life(BatchArgs B, const uint8_t *__restrict__ in,
                                                    uint8_t *__restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const uint64_t lo = B.total_cost * blockIdx.x / gridDim.x;
    const uint64_t hi = B.total_cost * (blockIdx.x + 1) / gridDim.x;
    // instance holding cost unit lo (uniform binary search)
    uint32_t a = 0, b = B.ninst;
    while (b - a > 1) {
        const uint32_t m = (a + b) / 2;
        if (B.cost_start[m] <= lo)
            a = m;
        else
            b = m;
    }
    uint32_t i = a;
    uint64_t j = 0;
    {
        const BatchInst &I = B.inst[i];
        j = (lo - I.cost_start + I.unit_cost - 1) / I.unit_cost;
    }
    int loaded = -1;  // expanded-tile configuration currently in LDS
    const XOp op{};
    while (i < B.ninst) {
        const BatchInst &I = B.inst[i];
        if (j >= I.units) {
            ++i;
            j = 0;
            continue;
        }
        if (I.cost_start + j * I.unit_cost >= hi) break;
        const uint8_t *ii = in + I.base;
        uint8_t *oo = out + I.base;
        __syncthreads();  // the previous unit's LDS reads are done
        switch (I.kind) {
        case kBX68:
        case kBX84:
        case kBXAny: {
            // this workgroup's run of consecutive tiles of the instance
            uint64_t je = (hi - I.cost_start + I.unit_cost - 1) / I.unit_cost;
            if (je > I.units) je = I.units;
            if constexpr (K > 1) {
                if (loaded != (int)I.xcfg) {
                    xtile_setupK<XLife>(I.xk, smem);
                    loaded = (int)I.xcfg;
                }
                if (I.xk.P == 88)
                    xtile_runK<XLife, 88, 16, 4, K>(I.xk, ii, oo, j, je, op, smem);
                else
                    xtile_runK<XLife, 0, 16, 4, K>(I.xk, ii, oo, j, je, op, smem);
                j = je;
                break;
            }
            const XLds<XLife> S(smem, I.x);
            if (loaded != (int)I.xcfg) {
                xtile_setup<XLife>(I.x, S);
                loaded = (int)I.xcfg;
            }
            if (I.kind == kBX84 && I.x.KM == 16 * 256 && I.x.R <= 2 * 256) {
                xtile_run<XLife, 84, 16, 2, true>(I.x, ii, oo, j, je, op, S);
            } else if (I.x.KM <= 16 * 256 && I.x.R <= 2 * 256) {
                if (I.kind == kBX84)
                    xtile_run<XLife, 84, 16, 2>(I.x, ii, oo, j, je, op, S);
                else if (I.kind == kBX68)
                    xtile_run<XLife, 68, 16, 2>(I.x, ii, oo, j, je, op, S);
                else
                    xtile_run<XLife, 0, 16, 2>(I.x, ii, oo, j, je, op, S);
            } else {
                for (uint64_t t = j; t < je; ++t) xtile_body<XLife, 0>(I.x, ii, oo, t, op, S);
            }
            j = je;
            break;
        }
        default:
            life_cell_unit(I.P, ii, oo, j);
            ++j;
            break;
        }
    }
}

// One group: instances of one tiled pattern, one workgroup per tile.
struct GroupArgs {
    const void *args;        // per instance: TileArgs or BitboxArgs
    const uint64_t *base;    // byte offset of each instance
    const uint64_t *tstart;  // ninst + 1 prefix sums of tile counts
    uint32_t ninst;
};

__device__ __forceinline__ uint32_t group_instance(const GroupArgs &G, uint64_t b)
{
    uint32_t a = 0, e = G.ninst;
    while (e - a > 1) {
        const uint32_t m = (a + e) / 2;
        if (G.tstart[m] <= b)
            a = m;
        else
            e = m;
    }
    return a;
}

template <class Pat, int K>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8)))
k_batch_tile(GroupArgs G, const uint8_t *__restrict__ in, uint8_t *__restrict__ out)
{
    using LDS = TileLds<Pat>;
    __shared__ uint32_t s_buf[3][LDS::WORDS];
    __shared__ __align__(16) uint32_t s_ring[kRingTab];
    const uint64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t i = group_instance(G, b);
    const TileArgs &A = reinterpret_cast<const TileArgs *>(G.args)[i];
    const uint64_t t = b - G.tstart[i], base = G.base[i];
    if constexpr (K == 1) {
        tile_body<Pat>(A, in + base, out + base, t, s_buf[0], s_buf[1]);
    } else {
        uint32_t *const buf[3] = {s_buf[0], s_buf[1], s_buf[2]};
        tile_bodyK<Pat, K>(A, in + base, out + base, t, buf, s_ring);
    }
}

template <class Pat, int K>
__global__ void __launch_bounds__(kBxThreads) __attribute__((amdgpu_waves_per_eu(6)))
k_batch_bitbox(GroupArgs G, const uint8_t *__restrict__ in, uint8_t *__restrict__ out)
{
    __shared__ uint32_t s_buf[2][kBxBuf];
    __shared__ uint64_t s_nb[9];
    __shared__ uint32_t s_ex;
    const uint64_t b = blockIdx.x;
    const uint32_t i = group_instance(G, b);
    const BitboxArgs &A = reinterpret_cast<const BitboxArgs *>(G.args)[i];
    const uint64_t base = G.base[i];
    bitbox_tile<Pat, K>(A, in + base, out + base, b - G.tstart[i], s_buf, s_nb, &s_ex);
}

// Instance of the persistent tiled launch (patterns with a tiled kernel).
struct TiledInst {
    uint32_t kind;        // kBTri, kBTriPaper, kBVicsek or kBBits
    uint32_t pad;
    uint64_t base;        // byte offset of the instance in the state buffer
    uint64_t units;       // tiles
    uint64_t unit_cells;  // cells per tile
    uint64_t cost_start;  // first cost unit (cell) of the instance
    TileArgs t;
    BitboxArgs x;
};

struct TiledArgs {
    const TiledInst *inst;
    const uint64_t *cost_start;  // ninst + 1 entries
    const uint64_t *tile_start;  // ninst + 1 prefix sums of tile counts
    const uint32_t *tile_map;    // workgroup-per-tile form: instance << 20 | tile, one entry per tile (or null)
    uint32_t ninst;
    uint64_t total_cost;
};

// LDS of a tile body: the bit-sliced layout (three state buffers, the ring
// tables 16-byte aligned) or the bit-row layout (two row buffers, nine
// bases, one flag word), whichever the kind uses; sizes in bytes.
template <class Pat>
__host__ __device__ constexpr size_t tiled_ring_offset()
{
    return (3 * (size_t)TileLds<Pat>::WORDS + 3) / 4 * 4;  // words
}
template <class Pat>
__host__ __device__ constexpr size_t tiled_lds_bytes()
{
    return (tiled_ring_offset<Pat>() + kRingTab) * 4;
}
constexpr size_t kBitsLds = 2 * (size_t)kBxBuf * 4 + 9 * 8 + 16;

template <class Pat, int K>
__device__ __forceinline__ void tiled_unit(const TileArgs &A, const uint8_t *in, uint8_t *out, uint64_t t,
                                           unsigned char *smem)
{
    using LDS = TileLds<Pat>;
    uint32_t *w = reinterpret_cast<uint32_t *>(smem);
    if constexpr (K == 1) {
        tile_body<Pat>(A, in, out, t, w, w + LDS::WORDS);
    } else {
        uint32_t *const buf[3] = {w, w + LDS::WORDS, w + 2 * LDS::WORDS};
        tile_bodyK<Pat, K>(A, in, out, t, buf, w + tiled_ring_offset<Pat>());
    }
}

template <int K>
__device__ __forceinline__ void bits_unit(const BitboxArgs &A, const uint8_t *in, uint8_t *out, uint64_t t,
                                          unsigned char *smem)
{
    if constexpr (K <= kBxMaxSteps) {
        uint32_t(*s_buf)[kBxBuf] = reinterpret_cast<uint32_t(*)[kBxBuf]>(smem);
        uint64_t *s_nb = reinterpret_cast<uint64_t *>(smem + ((2 * (size_t)kBxBuf * 4 + 7) & ~(size_t)7));
        bitbox_tile<PatCarpet, K>(A, in, out, t, s_buf, s_nb, reinterpret_cast<uint32_t *>(s_nb + 9));
    }
}

template <int K>
__device__ __forceinline__ void tiled_run(const TiledInst &I, const uint8_t *in, uint8_t *out, uint64_t j,
                                          unsigned char *smem)
{
    const uint8_t *ii = in + I.base;
    uint8_t *oo = out + I.base;
    switch (I.kind) {
    case kBTri: tiled_unit<PatTriangle, K>(I.t, ii, oo, j, smem); break;
    case kBTriPaper: tiled_unit<PatTrianglePaper, K>(I.t, ii, oo, j, smem); break;
    case kBVicsek: tiled_unit<PatVicsek, K>(I.t, ii, oo, j, smem); break;
    default: bits_unit<K>(I.x, ii, oo, j, smem); break;
    }
}

// K Life steps of every instance with a tiled kernel in one launch: the tiles
// of all such instances form one sequence, each run with its pattern's tile
// body (bit-sliced tiles of the triangle, its mirror image and the Vicsek
// cross; bit rows of the carpet).  Persistent (PerTile false): the sequence
// is weighted by cells and workgroup b takes the tiles whose first cell falls
// in the b-th equal share.  PerTile: one workgroup per tile, dealt to the
// XCDs in contiguous runs, eight waves per SIMD; the persistent form at six
// (its tile loop holds more registers).
template <int K, bool PerTile>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PerTile ? 8 : 6)))
k_batch_tiles(TiledArgs B, const uint8_t *__restrict__ in, uint8_t *__restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if constexpr (PerTile) {
        // one call site of the tile bodies (each inlined once: the kernel's
        // code must stay small enough for the instruction cache)
        const uint64_t b = xcd_remap(blockIdx.x, gridDim.x);
        uint32_t a = 0;
        uint64_t j;
        if (B.tile_map) {
            const uint32_t v = B.tile_map[b];
            a = v >> 20;
            j = v & 0xFFFFFu;
        } else {
            uint32_t e = B.ninst;
            while (e - a > 1) {
                const uint32_t m = (a + e) / 2;
                if (B.tile_start[m] <= b)
                    a = m;
                else
                    e = m;
            }
            j = b - B.tile_start[a];
        }
        tiled_run<K>(B.inst[a], in, out, j, smem);
        return;
    }
    const uint64_t lo = B.total_cost * blockIdx.x / gridDim.x;
    const uint64_t hi = B.total_cost * (blockIdx.x + 1) / gridDim.x;
    uint32_t a = 0, e = B.ninst;
    while (e - a > 1) {
        const uint32_t m = (a + e) / 2;
        if (B.cost_start[m] <= lo)
            a = m;
        else
            e = m;
    }
    uint32_t i = a;
    uint64_t j = 0;
    {
        const TiledInst &I = B.inst[i];
        j = (lo - I.cost_start + I.unit_cells - 1) / I.unit_cells;
    }
    while (i < B.ninst) {
        const TiledInst &I = B.inst[i];
        if (j >= I.units) {
            ++i;
            j = 0;
            continue;
        }
        if (I.cost_start + j * I.unit_cells >= hi) break;
        tiled_run<K>(I, in, out, j, smem);
        ++j;  // every tile body ends with a barrier: LDS is free for the next tile
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct BatchGroup {
    uint32_t kind;  // kBTri, kBTriPaper, kBVicsek or kBBits
    int K, K_max;   // steps per launch: chosen, most allowed
    std::vector<uint32_t> members;
    uint64_t ntiles;
    void *d_args;
    uint64_t *d_base, *d_tstart;
};

struct BatchHost {
    // instances with a tiled kernel run as one launch per pattern group
    // (tiled_form 0), one persistent launch over all of them (1) or one launch
    // over all of them with a workgroup per tile (2); the autotuner picks
    std::vector<BatchGroup> groups;
    int tiled_form;
    std::vector<TiledInst> tiled;
    TiledInst *d_tiled;
    uint64_t *d_tcost, *d_ttiles;
    uint32_t *d_tmap;  // tile order of the workgroup-per-tile form (null: instance order)
    uint64_t tcost_total, ttiles_total;
    size_t tlds;
    int Kt_max, Kt;             // steps per launch: most allowed, chosen
    unsigned twg, twg_max;      // workgroups per CU: chosen, most resident
    bool has_rest;  // instances for the persistent expanded-tile / thread-level launch
    int device;
    int cus;
    std::vector<BatchInst> inst;
    std::vector<uint64_t> offsets;  // byte offset of each instance; back() = total bytes
    std::vector<uint64_t> cells;
    uint64_t total_cells, total_bytes;
    BatchInst *d_inst;
    uint64_t *d_cost_start;
    uint64_t total_cost;
    unsigned xt_weight;  // cost per cell of the expanded-tile path (bit-sliced = 2, thread-level = 32)
    size_t lds, ldsk;  // dynamic LDS of the one-step and the K-step kernel
    int K;              // steps per launch of batch runs (1: one-step only)
    unsigned wg_per_cu, max_wg_per_cu;
    std::string key;
    hipStream_t cap;
    hipGraphExec_t gexec;
    const void *g_a, *g_b;
    int32_t g_steps;
    void *g_stream;
};

static std::mutex g_tune_mu;
struct TuneResult {
    unsigned wg, xt_weight, twg;
    int Kt;
    int tiled_form;
    std::vector<int> group_K;
};
static std::map<std::string, TuneResult> g_tune_cache;  // batch composition -> tuned launch shapes

const FractalHost &fractal_host_of(const sqz_fractal *f);  // api.hip

static uint32_t kind_of(const FractalHost &F)
{
    if (F.bitbox) return kBBits;
    if (F.tile_kind == 1) return kBTri;
    if (F.tile_kind == 2) return kBTriPaper;
    if (F.tile_kind == 3) return kBVicsek;
    if (F.xtile) return F.xtile->P == 84 ? kBX84 : (F.xtile->P == 68 ? kBX68 : kBXAny);
    return kBCell;
}

static bool grouped(uint32_t kind) { return kind == kBTri || kind == kBTriPaper || kind == kBVicsek || kind == kBBits; }

// Cost of a cell per path of the persistent launch (for its static split):
// expanded tile xt_weight (tuned), thread-level 32; grouped instances have no
// units there.  Uploads the instances and prefix sums.
static hipError_t upload_costs(BatchHost *H)
{
    const size_t n = H->inst.size();
    std::vector<uint64_t> cs(n + 1);
    uint64_t c = 0;
    for (size_t i = 0; i < n; ++i) {
        BatchInst &I = H->inst[i];
        const uint32_t k = I.kind;
        const uint64_t w = k == kBCell ? 32 : H->xt_weight;
        I.cost_start = c;
        I.unit_cost = I.unit_cells * w;
        cs[i] = c;
        c += I.units * I.unit_cost;
    }
    cs[n] = c;
    H->total_cost = c;
    hipError_t e = hipMemcpy(H->d_inst, H->inst.data(), sizeof(BatchInst) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(H->d_cost_start, cs.data(), sizeof(uint64_t) * (n + 1), hipMemcpyHostToDevice);
    return e;
}

sqz_status batch_create(const sqz_fractal *const *fr, int32_t count, BatchHost **out)
{
    BatchHost *H = new BatchHost();
    H->inst.resize(count);
    H->offsets.resize(count + 1);
    H->cells.resize(count);
    hipError_t e = hipGetDevice(&H->device);
    if (e != hipSuccess) {
        delete H;
        return hip_error(e, "hipGetDevice");
    }
    hipDeviceProp_t prop;
    H->cus = hipGetDeviceProperties(&prop, H->device) == hipSuccess ? prop.multiProcessorCount : 256;
    H->Kt_max = kMaxSteps;
    std::map<std::string, uint32_t> xcfg_ids;
    std::vector<uint64_t> cell_start(count + 1);
    uint64_t off = 0, cstart = 0;
    size_t lds = 0, ldsk = 0;
    int kmin = kMaxSteps;
    char buf[64];
    for (int32_t i = 0; i < count; ++i) {
        const FractalHost &F = fractal_host_of(fr[i]);
        if (F.device != H->device) {
            delete H;
            return set_error(SQZ_ERR_INVALID, "instance %d lives on device %d, not %d", i, F.device, H->device);
        }
        BatchInst &I = H->inst[i];
        memset(&I, 0, sizeof I);
        I.kind = kind_of(F);
        I.base = off;
        I.cells = F.N;
        I.cell_start = cstart;
        I.P = F.P;
        if (grouped(I.kind)) {
            TiledInst T;
            memset(&T, 0, sizeof T);
            T.kind = I.kind;
            T.base = off;
            if (I.kind == kBBits) {
                T.x = bitbox_args(F);
                T.units = T.x.ntiles;
                T.unit_cells = T.x.tile;
                H->Kt_max = std::min(H->Kt_max, bitbox_steps_per_launch(F));
                H->tlds = std::max(H->tlds, kBitsLds);
            } else {
                T.t = tile_args(F);
                T.units = T.t.ntiles;
                T.unit_cells = T.t.tile;
                H->Kt_max = std::min(H->Kt_max, tile_steps_per_launch(F));
                H->tlds = std::max(H->tlds, I.kind == kBVicsek ? tiled_lds_bytes<PatVicsek>()
                                                                : tiled_lds_bytes<PatTriangle>());
            }
            T.cost_start = H->tcost_total;
            H->tcost_total += T.units * T.unit_cells;
            H->tiled.push_back(T);
            BatchGroup *G = nullptr;
            for (BatchGroup &g : H->groups)
                if (g.kind == I.kind) G = &g;
            if (!G) {
                H->groups.push_back(BatchGroup{I.kind, kMaxSteps, kMaxSteps, {}, 0, nullptr, nullptr, nullptr});
                G = &H->groups.back();
            }
            G->members.push_back((uint32_t)i);
            G->K_max = std::min(G->K_max, I.kind == kBBits ? bitbox_steps_per_launch(F) : tile_steps_per_launch(F));
            G->K = G->K_max;
            I.units = 0;  // not in the expanded-tile / thread-level launch
            I.unit_cells = 1;
        } else if (I.kind != kBCell) {
            const XTileConfig *X = F.xtile;
            I.x = X->base;
            const size_t need = xt_layout(X->P, X->KM, X->R, 1, false, true, &I.x);
            I.x.vec = (X->KM % 16 == 0) ? 1u : 0u;
            lds = std::max(lds, need);
            if (X->K >= 2) {
                I.xk = X->kbase;
                ldsk = std::max(ldsk, xt_layoutK(I.xk.P, I.xk.rows, I.xk.KM, I.xk.R, 1, true, &I.xk));
                kmin = std::min(kmin, (int)X->K);
            } else {
                kmin = 1;
            }
            std::string key = std::to_string(F.s) + ":" + std::to_string(X->M);
            for (int j = 0; j < F.k; ++j) key += "," + std::to_string(F.ox[j]) + "/" + std::to_string(F.oy[j]);
            auto it = xcfg_ids.find(key);
            if (it == xcfg_ids.end()) it = xcfg_ids.emplace(key, (uint32_t)xcfg_ids.size()).first;
            I.xcfg = it->second;
            // tables are identical for one (pattern, M): use the first instance's copy
            for (int32_t p = 0; p < i; ++p)
                if ((H->inst[p].kind == I.kind) && H->inst[p].xcfg == I.xcfg && H->inst[p].kind != kBCell &&
                    H->inst[p].kind >= kBX68) {
                    I.x.lam = H->inst[p].x.lam;
                    I.x.ent = H->inst[p].x.ent;
                    I.x.rpos = H->inst[p].x.rpos;
                    I.x.rinfo = H->inst[p].x.rinfo;
                    break;
                }
            I.units = X->ntiles;
            I.unit_cells = X->KM;
            H->has_rest = true;
        } else {
            I.units = (F.N + kCellUnit - 1) / kCellUnit;
            I.unit_cells = kCellUnit;
            kmin = 1;
            H->has_rest = true;
        }
        snprintf(buf, sizeof buf, "%d:%d:%d;", (int)I.kind, F.s, F.r);
        H->key += buf;
        H->cells[i] = F.N;
        cell_start[i] = cstart;
        H->offsets[i] = off;
        cstart += F.N;
        off += (F.N + 255) / 256 * 256;
    }
    cell_start[count] = cstart;
    H->offsets[count] = off;
    // The tiled launch forms take the instances in an order that spreads every
    // pattern kind evenly over the launch (each instance keyed by the middle
    // of its share of its kind's cells), so that the workgroups on the chip at
    // any time mix tile bodies that load different units (vector ALU, LDS,
    // memory); instances of one kind keep their relative order.
    if (SQZ_BATCH_INTERLEAVE) {
        std::map<uint32_t, uint64_t> kind_total, kind_seen;
        for (const TiledInst &T : H->tiled) kind_total[T.kind] += T.units * T.unit_cells;
        std::vector<std::pair<double, size_t>> key(H->tiled.size());
        for (size_t q = 0; q < H->tiled.size(); ++q) {
            const TiledInst &T = H->tiled[q];
            const uint64_t c = T.units * T.unit_cells;
            key[q] = {(kind_seen[T.kind] + 0.5 * (double)c) / (double)kind_total[T.kind], q};
            kind_seen[T.kind] += c;
        }
        std::stable_sort(key.begin(), key.end());
        std::vector<TiledInst> ord;
        ord.reserve(H->tiled.size());
        for (const auto &k : key) ord.push_back(H->tiled[k.second]);
        H->tiled.swap(ord);
        H->tcost_total = 0;
        for (TiledInst &T : H->tiled) {
            T.cost_start = H->tcost_total;
            H->tcost_total += T.units * T.unit_cells;
        }
    }
    H->total_cells = cstart;
    H->total_bytes = off;
    H->lds = std::max<size_t>(lds, 16);
    H->K = H->has_rest && kmin >= 2 ? std::min(kmin, 3) : 1;
    H->ldsk = std::max<size_t>(ldsk, 16);
    H->d_inst = nullptr;
    H->d_cost_start = nullptr;
    H->cap = nullptr;
    H->gexec = nullptr;
    e = hipMalloc(&H->d_inst, sizeof(BatchInst) * count);
    if (e == hipSuccess) e = hipMalloc(&H->d_cost_start, sizeof(uint64_t) * (count + 1));
    // the persistent tiled launch: instances and cost prefix sums
    if (e == hipSuccess && !H->tiled.empty()) {
        const size_t m = H->tiled.size();
        std::vector<uint64_t> cs(m + 1);
        std::vector<uint64_t> ts(m + 1);
        for (size_t q = 0; q < m; ++q) {
            cs[q] = H->tiled[q].cost_start;
            ts[q] = H->ttiles_total;
            H->ttiles_total += H->tiled[q].units;
        }
        cs[m] = H->tcost_total;
        ts[m] = H->ttiles_total;
        e = hipMalloc(&H->d_tiled, sizeof(TiledInst) * m);
        if (e == hipSuccess) e = hipMemcpy(H->d_tiled, H->tiled.data(), sizeof(TiledInst) * m, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&H->d_tcost, sizeof(uint64_t) * (m + 1));
        if (e == hipSuccess) e = hipMemcpy(H->d_tcost, cs.data(), sizeof(uint64_t) * (m + 1), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&H->d_ttiles, sizeof(uint64_t) * (m + 1));
        if (e == hipSuccess) e = hipMemcpy(H->d_ttiles, ts.data(), sizeof(uint64_t) * (m + 1), hipMemcpyHostToDevice);
        // workgroup-per-tile order: the tiles of every pattern kind spread evenly over
        // the launch, each tile keyed by the middle of its place among its kind's tiles
        H->d_tmap = nullptr;
        bool fits = m < 4096;
        for (size_t q = 0; q < m && fits; ++q) fits = H->tiled[q].units <= 0xFFFFFu;
        if (e == hipSuccess && fits && SQZ_BATCH_TILE_MAP) {
            std::map<uint32_t, uint64_t> kind_tiles, kind_seen;
            for (const TiledInst &T : H->tiled) kind_tiles[T.kind] += T.units;
            std::vector<std::pair<double, uint32_t>> key;
            key.reserve(H->ttiles_total);
            for (size_t q = 0; q < m; ++q) {
                const TiledInst &T = H->tiled[q];
                const double n = (double)kind_tiles[T.kind];
                for (uint64_t j = 0; j < T.units; ++j)
                    key.push_back({((double)kind_seen[T.kind]++ + 0.5) / n, (uint32_t)(q << 20 | j)});
            }
            std::stable_sort(key.begin(), key.end(),
                             [](const std::pair<double, uint32_t> &x, const std::pair<double, uint32_t> &y) {
                                 return x.first < y.first;
                             });
            std::vector<uint32_t> map(key.size());
            for (size_t i = 0; i < key.size(); ++i) map[i] = key[i].second;
            e = hipMalloc(&H->d_tmap, sizeof(uint32_t) * map.size());
            if (e == hipSuccess)
                e = hipMemcpy(H->d_tmap, map.data(), sizeof(uint32_t) * map.size(), hipMemcpyHostToDevice);
        }
        H->Kt = H->Kt_max;
        int per_cu = 0;
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_tiles<2, false>, 256, H->tlds);
        H->twg_max = per_cu < 1 ? 1u : (unsigned)per_cu;
        H->twg = H->twg_max;
    }
    // groups: per-instance kernel arguments, bases and tile prefix sums
    for (size_t g = 0; g < H->groups.size() && e == hipSuccess; ++g) {
        BatchGroup &G = H->groups[g];
        const size_t m = G.members.size();
        const bool bits = G.kind == kBBits;
        std::vector<TileArgs> ta(bits ? 0 : m);
        std::vector<BitboxArgs> ba(bits ? m : 0);
        std::vector<uint64_t> base(m), ts(m + 1);
        uint64_t tiles = 0;
        for (size_t q = 0; q < m; ++q) {
            const FractalHost &F = fractal_host_of(fr[G.members[q]]);
            ts[q] = tiles;
            base[q] = H->offsets[G.members[q]];
            if (bits) {
                ba[q] = bitbox_args(F);
                tiles += ba[q].ntiles;
            } else {
                ta[q] = tile_args(F);
                tiles += ta[q].ntiles;
            }
        }
        ts[m] = tiles;
        G.ntiles = tiles;
        const size_t asz = bits ? sizeof(BitboxArgs) * m : sizeof(TileArgs) * m;
        e = hipMalloc(&G.d_args, asz);
        if (e == hipSuccess) e = hipMemcpy(G.d_args, bits ? (const void *)ba.data() : (const void *)ta.data(), asz,
                                           hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&G.d_base, sizeof(uint64_t) * m);
        if (e == hipSuccess) e = hipMemcpy(G.d_base, base.data(), sizeof(uint64_t) * m, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&G.d_tstart, sizeof(uint64_t) * (m + 1));
        if (e == hipSuccess) e = hipMemcpy(G.d_tstart, ts.data(), sizeof(uint64_t) * (m + 1), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMalloc(&H->d_cost_start, sizeof(uint64_t) * (count + 1));
    H->xt_weight = 4;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(H->key);
        if (it != g_tune_cache.end()) {
            H->xt_weight = it->second.xt_weight;
            if (!H->tiled.empty()) {
                H->twg = std::min(it->second.twg, H->twg_max);
                H->Kt = std::min(it->second.Kt, H->Kt_max);
                H->tiled_form = it->second.tiled_form;
                for (size_t g = 0; g < H->groups.size() && g < it->second.group_K.size(); ++g)
                    H->groups[g].K = std::min(it->second.group_K[g], H->groups[g].K_max);
            }
        }
    }
    if (e == hipSuccess) e = upload_costs(H);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&H->cap, hipStreamNonBlocking);
    int per_cu = 0;
    if (e == hipSuccess) {
        switch (H->K) {
        case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_life<3>, 256, H->ldsk); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_life<2>, 256, H->ldsk); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_life<1>, 256, H->lds); break;
        }
    }
    if (e != hipSuccess) {
        batch_destroy(H);
        return hip_error(e, "batch setup");
    }
    H->max_wg_per_cu = per_cu < 1 ? 1u : (unsigned)per_cu;
    H->wg_per_cu = H->max_wg_per_cu;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(H->key);
        if (it != g_tune_cache.end()) H->wg_per_cu = std::min(it->second.wg, H->max_wg_per_cu);
    }
    *out = H;
    return SQZ_OK;
}

void batch_destroy(BatchHost *H)
{
    if (!H) return;
    if (H->gexec) (void)hipGraphExecDestroy(H->gexec);
    if (H->cap) (void)hipStreamDestroy(H->cap);
    (void)hipFree(H->d_inst);
    (void)hipFree(H->d_cost_start);
    (void)hipFree(H->d_tiled);
    (void)hipFree(H->d_tcost);
    (void)hipFree(H->d_ttiles);
    if (H->d_tmap) (void)hipFree(H->d_tmap);
    for (BatchGroup &G : H->groups) {
        (void)hipFree(G.d_args);
        (void)hipFree(G.d_base);
        (void)hipFree(G.d_tstart);
    }
    delete H;
}

// One launch of `steps` (1..H->K) steps.
static sqz_status launch_batch(const BatchHost *H, unsigned wg_per_cu, const uint8_t *in, uint8_t *out, int steps,
                               hipStream_t st)
{
    BatchArgs A;
    A.inst = H->d_inst;
    A.cost_start = H->d_cost_start;
    A.ninst = (uint32_t)H->inst.size();
    A.total_cost = H->total_cost;
    uint64_t grid = (uint64_t)H->cus * wg_per_cu;
    if (grid < 1) grid = 1;
    switch (steps) {
    case 3: hipLaunchKernelGGL(k_batch_life<3>, dim3((unsigned)grid), dim3(256), H->ldsk, st, A, in, out); break;
    case 2: hipLaunchKernelGGL(k_batch_life<2>, dim3((unsigned)grid), dim3(256), H->ldsk, st, A, in, out); break;
    default: hipLaunchKernelGGL(k_batch_life<1>, dim3((unsigned)grid), dim3(256), H->lds, st, A, in, out); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "batch launch");
}

template <class Pat>
static void launch_tile_group(const GroupArgs &A, unsigned grid, const uint8_t *in, uint8_t *out, int steps,
                              hipStream_t st)
{
    switch (steps) {
    case 1: hipLaunchKernelGGL((k_batch_tile<Pat, 1>), dim3(grid), dim3(kBlock), 0, st, A, in, out); break;
    case 2: hipLaunchKernelGGL((k_batch_tile<Pat, 2>), dim3(grid), dim3(kBlock), 0, st, A, in, out); break;
    case 3: hipLaunchKernelGGL((k_batch_tile<Pat, 3>), dim3(grid), dim3(kBlock), 0, st, A, in, out); break;
    case 4: hipLaunchKernelGGL((k_batch_tile<Pat, 4>), dim3(grid), dim3(kBlock), 0, st, A, in, out); break;
    case 5: hipLaunchKernelGGL((k_batch_tile<Pat, 5>), dim3(grid), dim3(kBlock), 0, st, A, in, out); break;
    case 6: hipLaunchKernelGGL((k_batch_tile<Pat, 6>), dim3(grid), dim3(kBlock), 0, st, A, in, out); break;
    case 7: hipLaunchKernelGGL((k_batch_tile<Pat, 7>), dim3(grid), dim3(kBlock), 0, st, A, in, out); break;
    case 8: hipLaunchKernelGGL((k_batch_tile<Pat, 8>), dim3(grid), dim3(kBlock), 0, st, A, in, out); break;
    case 9: hipLaunchKernelGGL((k_batch_tile<Pat, 9>), dim3(grid), dim3(kBlock), 0, st, A, in, out); break;
    default: hipLaunchKernelGGL((k_batch_tile<Pat, 10>), dim3(grid), dim3(kBlock), 0, st, A, in, out); break;
    }
}

static void launch_bits_group(const GroupArgs &A, unsigned grid, const uint8_t *in, uint8_t *out, int steps,
                              hipStream_t st)
{
    const dim3 g(grid), b(kBxThreads);
    switch (steps) {
    case 1: hipLaunchKernelGGL((k_batch_bitbox<PatCarpet, 1>), g, b, 0, st, A, in, out); break;
    case 2: hipLaunchKernelGGL((k_batch_bitbox<PatCarpet, 2>), g, b, 0, st, A, in, out); break;
    case 3: hipLaunchKernelGGL((k_batch_bitbox<PatCarpet, 3>), g, b, 0, st, A, in, out); break;
    case 4: hipLaunchKernelGGL((k_batch_bitbox<PatCarpet, 4>), g, b, 0, st, A, in, out); break;
    case 5: hipLaunchKernelGGL((k_batch_bitbox<PatCarpet, 5>), g, b, 0, st, A, in, out); break;
    case 6: hipLaunchKernelGGL((k_batch_bitbox<PatCarpet, 6>), g, b, 0, st, A, in, out); break;
    case 7: hipLaunchKernelGGL((k_batch_bitbox<PatCarpet, 7>), g, b, 0, st, A, in, out); break;
    case 8: hipLaunchKernelGGL((k_batch_bitbox<PatCarpet, 8>), g, b, 0, st, A, in, out); break;
    case 9: hipLaunchKernelGGL((k_batch_bitbox<PatCarpet, 9>), g, b, 0, st, A, in, out); break;
    default: hipLaunchKernelGGL((k_batch_bitbox<PatCarpet, 10>), g, b, 0, st, A, in, out); break;
    }
}

// One launch of `steps` (1..G.K) steps for every instance of group G.
static sqz_status launch_group(const BatchGroup &G, const uint8_t *in, uint8_t *out, int steps, hipStream_t st)
{
    const GroupArgs A{G.d_args, G.d_base, G.d_tstart, (uint32_t)G.members.size()};
    const unsigned grid = (unsigned)G.ntiles;
    switch (G.kind) {
    case kBTri: launch_tile_group<PatTriangle>(A, grid, in, out, steps, st); break;
    case kBTriPaper: launch_tile_group<PatTrianglePaper>(A, grid, in, out, steps, st); break;
    case kBVicsek: launch_tile_group<PatVicsek>(A, grid, in, out, steps, st); break;
    default: launch_bits_group(A, grid, in, out, steps, st); break;
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "batch group launch");
}

template <bool PerTile>
static void launch_tiles_k(int steps, dim3 g, dim3 b, size_t L, hipStream_t st, const TiledArgs &A, const uint8_t *in,
                           uint8_t *out)
{
    switch (steps) {
    case 1: hipLaunchKernelGGL((k_batch_tiles<1, PerTile>), g, b, L, st, A, in, out); break;
    case 2: hipLaunchKernelGGL((k_batch_tiles<2, PerTile>), g, b, L, st, A, in, out); break;
    case 3: hipLaunchKernelGGL((k_batch_tiles<3, PerTile>), g, b, L, st, A, in, out); break;
    case 4: hipLaunchKernelGGL((k_batch_tiles<4, PerTile>), g, b, L, st, A, in, out); break;
    case 5: hipLaunchKernelGGL((k_batch_tiles<5, PerTile>), g, b, L, st, A, in, out); break;
    case 6: hipLaunchKernelGGL((k_batch_tiles<6, PerTile>), g, b, L, st, A, in, out); break;
    case 7: hipLaunchKernelGGL((k_batch_tiles<7, PerTile>), g, b, L, st, A, in, out); break;
    case 8: hipLaunchKernelGGL((k_batch_tiles<8, PerTile>), g, b, L, st, A, in, out); break;
    case 9: hipLaunchKernelGGL((k_batch_tiles<9, PerTile>), g, b, L, st, A, in, out); break;
    default: hipLaunchKernelGGL((k_batch_tiles<10, PerTile>), g, b, L, st, A, in, out); break;
    }
}

// One launch of `steps` (1..H->Kt_max) steps for every tiled instance: form 1
// persistent (wg_per_cu workgroups per CU), form 2 one workgroup per tile.
static sqz_status launch_tiled(const BatchHost *H, int form, unsigned wg_per_cu, const uint8_t *in, uint8_t *out,
                               int steps, hipStream_t st)
{
    TiledArgs A;
    A.inst = H->d_tiled;
    A.cost_start = H->d_tcost;
    A.tile_start = H->d_ttiles;
    A.tile_map = H->d_tmap;
    A.ninst = (uint32_t)H->tiled.size();
    A.total_cost = H->tcost_total;
    uint64_t grid = form == 2 ? H->ttiles_total : (uint64_t)H->cus * wg_per_cu;
    if (grid < 1) grid = 1;
    if (grid > 0xFFFFFFFFull) return set_error(SQZ_ERR_RANGE, "%llu tiles exceed one launch", (unsigned long long)grid);
    const dim3 g((unsigned)grid), b(256);
    const size_t L = H->tlds;
    if (form == 2)
        launch_tiles_k<true>(steps, g, b, L, st, A, in, out);
    else
        launch_tiles_k<false>(steps, g, b, L, st, A, in, out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "batch tiled launch");
}

// All launches of `steps` steps: the tiled launch and the expanded-tile /
// thread-level launch follow their own plans (each with the parity of
// `steps`, so every result lands in the same buffer).
static sqz_status launch_all(const BatchHost *H, const uint8_t *a, const uint8_t *b, int32_t steps, hipStream_t st)
{
    sqz_status s2 = SQZ_OK;
    uint8_t *const A = const_cast<uint8_t *>(a), *const B = const_cast<uint8_t *>(b);
    if (!H->tiled.empty() && H->tiled_form != 0) {
        const std::vector<int> plan = plan_launches(steps, H->Kt);
        for (size_t i = 0; i < plan.size() && s2 == SQZ_OK; ++i)
            s2 = launch_tiled(H, H->tiled_form, H->twg, (i & 1) ? B : A, (i & 1) ? A : B, plan[i], st);
    } else {
        for (size_t g = 0; g < H->groups.size() && s2 == SQZ_OK; ++g) {
            const std::vector<int> plan = plan_launches(steps, H->groups[g].K);
            for (size_t i = 0; i < plan.size() && s2 == SQZ_OK; ++i)
                s2 = launch_group(H->groups[g], (i & 1) ? B : A, (i & 1) ? A : B, plan[i], st);
        }
    }
    if (H->has_rest) {
        const std::vector<int> plan = plan_launches(steps, H->K);
        for (size_t i = 0; i < plan.size() && s2 == SQZ_OK; ++i)
            s2 = launch_batch(H, H->wg_per_cu, (i & 1) ? B : A, (i & 1) ? A : B, plan[i], st);
    }
    return s2;
}

sqz_status batch_step(const BatchHost *H, const uint8_t *in, uint8_t *out, hipStream_t st)
{
    return launch_all(H, in, out, 1, st);
}

sqz_status batch_run(BatchHost *H, uint8_t *a, uint8_t *b, int32_t steps, hipStream_t st)
{
    if (steps == 0) return SQZ_OK;
    if (steps == 1) return batch_step(H, a, b, st);
    if (!(H->gexec && H->g_a == a && H->g_b == b && H->g_steps == steps)) {
        if (H->gexec) {
            (void)hipGraphExecDestroy(H->gexec);
            H->gexec = nullptr;
        }
        hipError_t e = hipStreamBeginCapture(H->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
        const sqz_status s2 = launch_all(H, a, b, steps, H->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(H->cap, &g);
        if (s2 != SQZ_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s2;
        }
        if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&H->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            H->gexec = nullptr;
            return hip_error(e, "hipGraphInstantiate");
        }
        H->g_a = a;
        H->g_b = b;
        H->g_steps = steps;
    }
    hipError_t e = hipGraphLaunch(H->gexec, st);
    return e == hipSuccess ? SQZ_OK : hip_error(e, "hipGraphLaunch");
}

// Milliseconds of `launches` of the given shape on the caller's buffers.
template <class F>
static sqz_status time_launches(hipStream_t st, hipEvent_t e0, hipEvent_t e1, F &&launch_i, int launches, float *ms)
{
    sqz_status st2 = launch_i(0);  // warm-up
    if (st2 != SQZ_OK) return st2;
    (void)hipEventRecord(e0, st);
    for (int i = 0; i < launches && st2 == SQZ_OK; ++i) st2 = launch_i(i);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) return set_error(SQZ_ERR_HIP, "autotune synchronisation failed");
    (void)hipEventElapsedTime(ms, e0, e1);
    return st2;
}

sqz_status batch_autotune(BatchHost *H, uint8_t *a, uint8_t *b, hipStream_t st, unsigned *best_out)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_error(SQZ_ERR_HIP, "hipEventCreate failed");
    sqz_status st2 = SQZ_OK;
    // (1) the tiled instances, each candidate timed per step over four
    // launches of its steps per launch: one launch per pattern group (steps
    // per launch per group), against one persistent launch (workgroups per CU
    // x steps per launch)
    if (!H->tiled.empty()) {
        const int ks[] = {1, 2, 3, 4, 5, 6, 8, 10};
        float grouped_ms = 0.0f;
        for (BatchGroup &G : H->groups) {
            float best_ms = 1e30f;
            int bk = G.K;
            for (int K : ks) {
                if (K > G.K_max || (K == 1 && G.K_max > 1) || st2 != SQZ_OK) continue;
                float ms = 0.0f;
                st2 = time_launches(st, e0, e1, [&](int i) {
                    return launch_group(G, (i & 1) ? b : a, (i & 1) ? a : b, K, st);
                }, 4, &ms);
                ms /= 4.0f * K;
                if (st2 == SQZ_OK && ms < best_ms) {
                    best_ms = ms;
                    bk = K;
                }
            }
            G.K = bk;
            grouped_ms += best_ms;
        }
        // one launch over all tiled instances: a workgroup per tile (w = 0), or
        // persistent with w workgroups per CU
        const unsigned ws[] = {0, 2, 3, 4, 5, 6, 8};
        float best_ms = 1e30f;
        unsigned bw = H->twg;
        int bk = H->Kt, bf = 2;
        for (int K : ks) {
            if (K > H->Kt_max || (K == 1 && H->Kt_max > 1)) continue;
            for (unsigned w : ws) {
                if (w > H->twg_max || st2 != SQZ_OK) continue;
                const int form = w == 0 ? 2 : 1;
                float ms = 0.0f;
                st2 = time_launches(st, e0, e1, [&](int i) {
                    return launch_tiled(H, form, w, (i & 1) ? b : a, (i & 1) ? a : b, K, st);
                }, 4, &ms);
                ms /= 4.0f * K;
                if (st2 == SQZ_OK && ms < best_ms) {
                    best_ms = ms;
                    bf = form;
                    if (w) bw = w;
                    bk = K;
                }
            }
        }
        H->twg = bw;
        H->Kt = bk;
        H->tiled_form = best_ms < grouped_ms ? bf : 0;
    }
    // (2) the expanded-tile / thread-level launch: workgroups per CU x the
    // expanded-tile cost weight
    if (H->has_rest && st2 == SQZ_OK) {
        bool has_xt = false;
        for (const BatchInst &I : H->inst) has_xt |= I.kind >= kBX68 && I.kind <= kBXAny;
        const unsigned weights[] = {2, 3, 4, 6, 8};
        unsigned best = H->wg_per_cu, best_w = H->xt_weight;
        float best_ms = 1e30f;
        for (unsigned wi = 0; wi < (has_xt ? 5u : 1u) && st2 == SQZ_OK; ++wi) {
            if (has_xt) {
                H->xt_weight = weights[wi];
                hipError_t e = upload_costs(H);
                if (e != hipSuccess) {
                    st2 = hip_error(e, "batch cost upload");
                    break;
                }
            }
            for (unsigned w = 1; w <= H->max_wg_per_cu && st2 == SQZ_OK; w = (w < 4 ? w + 1 : w * 2)) {
                float ms = 0.0f;
                st2 = time_launches(st, e0, e1, [&](int i) {
                    return launch_batch(H, w, (i & 1) ? b : a, (i & 1) ? a : b, H->K, st);
                }, 4, &ms);
                if (st2 == SQZ_OK && ms < best_ms) {
                    best_ms = ms;
                    best = w;
                    best_w = H->xt_weight;
                }
            }
        }
        H->xt_weight = best_w;
        hipError_t e = upload_costs(H);
        if (st2 == SQZ_OK && e != hipSuccess) st2 = hip_error(e, "batch cost upload");
        H->wg_per_cu = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st2 != SQZ_OK) return st2;
    if (H->gexec) {
        (void)hipGraphExecDestroy(H->gexec);
        H->gexec = nullptr;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        std::vector<int> gk;
        for (const BatchGroup &G : H->groups) gk.push_back(G.K);
        g_tune_cache[H->key] = TuneResult{H->wg_per_cu, H->xt_weight, H->twg, H->Kt, H->tiled_form, gk};
    }
    if (best_out) *best_out = H->tiled.empty() ? H->wg_per_cu : H->twg;
    return SQZ_OK;
}

sqz_status batch_set_tiled(BatchHost *H, int32_t persistent, int32_t steps_per_launch, int32_t wg_per_cu)
{
    if (persistent < 0 || persistent > 2) return set_error(SQZ_ERR_INVALID, "launch form %d outside 0..2", persistent);
    if (steps_per_launch < 0 || (steps_per_launch > 0 && (H->tiled.empty() || steps_per_launch > H->Kt_max)))
        return set_error(SQZ_ERR_INVALID, "steps_per_launch %d outside 0..%d", steps_per_launch,
                         H->tiled.empty() ? 0 : H->Kt_max);
    if (wg_per_cu < 0 || (wg_per_cu > 0 && (H->tiled.empty() || (unsigned)wg_per_cu > H->twg_max)))
        return set_error(SQZ_ERR_INVALID, "wg_per_cu %d outside 0..%u", wg_per_cu, H->tiled.empty() ? 0u : H->twg_max);
    H->tiled_form = persistent;
    if (steps_per_launch > 0) {
        H->Kt = steps_per_launch;
        for (BatchGroup &G : H->groups) G.K = std::min(steps_per_launch, G.K_max);
    }
    if (wg_per_cu > 0) H->twg = (unsigned)wg_per_cu;
    if (H->gexec) {
        (void)hipGraphExecDestroy(H->gexec);
        H->gexec = nullptr;
    }
    return SQZ_OK;
}

uint64_t batch_total_bytes(const BatchHost *H) { return H->total_bytes; }
uint64_t batch_offset(const BatchHost *H, int32_t i) { return H->offsets[i]; }
int32_t batch_count(const BatchHost *H) { return (int32_t)H->inst.size(); }
unsigned batch_wg_per_cu(const BatchHost *H) { return H->wg_per_cu; }
int batch_steps_per_launch(const BatchHost *H)
{
    int k = H->has_rest ? H->K : kMaxSteps;
    if (!H->tiled.empty() && H->tiled_form != 0)
        k = std::min(k, H->Kt);
    else
        for (const BatchGroup &G : H->groups) k = std::min(k, G.K);
    return k < 1 ? 1 : k;
}
uint64_t batch_total_cells(const BatchHost *H) { return H->total_cells; }
void batch_tiled_form(const BatchHost *H, int32_t *form, int32_t *steps_per_launch, int32_t *wg_per_cu)
{
    *form = H->tiled.empty() ? -1 : H->tiled_form;
    *steps_per_launch = H->tiled.empty() ? 0 : H->Kt;
    *wg_per_cu = H->tiled.empty() || H->tiled_form != 1 ? 0 : (int32_t)H->twg;
}

}  // namespace sqz
