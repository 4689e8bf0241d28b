// Batched Life: many independent fractals of mixed replica pattern and level
// advanced together, one persistent launch per step.
//
// Every instance owns a 256-byte aligned range of one state buffer.  Its work
// is a list of units: level-M tiles for the bit-sliced (triangle, Vicsek) and
// expanded-tile (any pattern) paths, runs of 4096 cells for the thread-level
// path (instances too small to tile).  The units of all instances form one
// sequence; workgroup b takes the units whose first cell falls in the b-th
// equal share of all cells, so the split is balanced by cells and each
// workgroup walks adjacent tiles of one or two instances.  The tile bodies are
// the same device functions the single-fractal kernels use, with LDS carved
// from one dynamic buffer; the expanded-tile tables are reloaded only when a
// workgroup moves to an instance with a different tile configuration.
//
// Runs of several steps are captured once into a hipGraph (kernel nodes only)
// and replayed; an autotuner times candidate grid sizes on the caller's
// buffers and keeps the fastest, cached per batch composition.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tile_device.h"
#include "xtile_device.h"

struct sqz_fractal;  // api.hip

namespace sqz {

enum BatchKind : uint32_t { kBTri = 1, kBTriPaper = 2, kBVicsek = 3, kBX68 = 4, kBX84 = 5, kBXAny = 6, kBCell = 7 };

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

// LDS word offset of the ring tables in the multi-step layout (16-byte aligned)
template <class Pat>
__host__ __device__ constexpr int ring_tab_offset()
{
    return (3 * TileLds<Pat>::WORDS + 3) / 4 * 4;
}

template <class Pat, int K>
__device__ __forceinline__ void bitsliced_unit(const BatchInst &I, const uint8_t *in, uint8_t *out, uint64_t t,
                                               unsigned char *smem)
{
    using LDS = TileLds<Pat>;
    uint32_t *s_in = reinterpret_cast<uint32_t *>(smem);
    if constexpr (K == 1) {
        tile_body<Pat>(I.tile, in, out, t, s_in, s_in + LDS::WORDS);
    } else {
        uint32_t *const buf[3] = {s_in, s_in + LDS::WORDS, s_in + 2 * LDS::WORDS};
        tile_bodyK<Pat, K>(I.tile, in, out, t, buf, s_in + ring_tab_offset<Pat>());
    }
}

// K Life steps of every instance (K > 1: every instance has multi-step tiles).
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
        case kBTri:
            loaded = -1;
            bitsliced_unit<PatTriangle, K>(I, ii, oo, j, smem);
            ++j;
            break;
        case kBTriPaper:
            loaded = -1;
            bitsliced_unit<PatTrianglePaper, K>(I, ii, oo, j, smem);
            ++j;
            break;
        case kBVicsek:
            loaded = -1;
            bitsliced_unit<PatVicsek, K>(I, ii, oo, j, smem);
            ++j;
            break;
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

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct BatchHost {
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
static std::map<std::string, std::pair<unsigned, unsigned>> g_tune_cache;  // key -> (wg per CU, xt weight)

const FractalHost &fractal_host_of(const sqz_fractal *f);  // api.hip

static uint32_t kind_of(const FractalHost &F)
{
    if (F.tile_kind == 1) return kBTri;
    if (F.tile_kind == 2) return kBTriPaper;
    if (F.tile_kind == 3) return kBVicsek;
    if (F.xtile) return F.xtile->P == 84 ? kBX84 : (F.xtile->P == 68 ? kBX68 : kBXAny);
    return kBCell;
}

template <class Pat>
static size_t tile_lds(bool multi)
{
    return multi ? (size_t)(ring_tab_offset<Pat>() + kRingTab) * 4 : (size_t)(2 * TileLds<Pat>::WORDS) * 4;
}

static size_t tile_lds_of(const FractalHost &F, bool multi)
{
    switch (F.tile_kind) {
    case 1: return tile_lds<PatTriangle>(multi);
    case 2: return tile_lds<PatTrianglePaper>(multi);
    default: return tile_lds<PatVicsek>(multi);
    }
}

// Cost of a cell per path (for the static split): bit-sliced 2, expanded tile
// xt_weight (tuned), thread-level 32.  Uploads the instances and prefix sums.
static hipError_t upload_costs(BatchHost *H)
{
    const size_t n = H->inst.size();
    std::vector<uint64_t> cs(n + 1);
    uint64_t c = 0;
    for (size_t i = 0; i < n; ++i) {
        BatchInst &I = H->inst[i];
        const uint32_t k = I.kind;
        const uint64_t w = (k == kBTri || k == kBTriPaper || k == kBVicsek) ? 2 : (k == kBCell ? 32 : H->xt_weight);
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
        if (I.kind == kBTri || I.kind == kBTriPaper || I.kind == kBVicsek) {
            I.tile = tile_args(F);
            I.units = I.tile.ntiles;
            I.unit_cells = I.tile.tile;
            lds = std::max(lds, tile_lds_of(F, false));
            ldsk = std::max(ldsk, tile_lds_of(F, true));
            kmin = std::min(kmin, tile_steps_per_launch(F));
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
                    I.x.mem_in = H->inst[p].x.mem_in;
                    I.x.rpos = H->inst[p].x.rpos;
                    I.x.rinfo = H->inst[p].x.rinfo;
                    break;
                }
            I.units = X->ntiles;
            I.unit_cells = X->KM;
        } else {
            I.units = (F.N + kCellUnit - 1) / kCellUnit;
            I.unit_cells = kCellUnit;
            kmin = 1;
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
    H->total_cells = cstart;
    H->total_bytes = off;
    H->lds = std::max<size_t>(lds, 16);
    H->K = count > 0 && kmin >= 2 ? std::min(kmin, 3) : 1;
    H->ldsk = std::max<size_t>(ldsk, 16);
    H->d_inst = nullptr;
    H->d_cost_start = nullptr;
    H->cap = nullptr;
    H->gexec = nullptr;
    e = hipMalloc(&H->d_inst, sizeof(BatchInst) * count);
    if (e == hipSuccess) e = hipMalloc(&H->d_cost_start, sizeof(uint64_t) * (count + 1));
    H->xt_weight = 4;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(H->key);
        if (it != g_tune_cache.end()) H->xt_weight = it->second.second;
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
        if (H->d_inst) (void)hipFree(H->d_inst);
        if (H->d_cost_start) (void)hipFree(H->d_cost_start);
        if (H->cap) (void)hipStreamDestroy(H->cap);
        delete H;
        return hip_error(e, "batch setup");
    }
    H->max_wg_per_cu = per_cu < 1 ? 1u : (unsigned)per_cu;
    H->wg_per_cu = H->max_wg_per_cu;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(H->key);
        if (it != g_tune_cache.end()) H->wg_per_cu = std::min(it->second.first, H->max_wg_per_cu);
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

sqz_status batch_step(const BatchHost *H, const uint8_t *in, uint8_t *out, hipStream_t st)
{
    return launch_batch(H, H->wg_per_cu, in, out, 1, st);
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
        sqz_status s2 = SQZ_OK;
        const std::vector<int> plan = plan_launches(steps, H->K);
        for (size_t i = 0; i < plan.size() && s2 == SQZ_OK; ++i)
            s2 = launch_batch(H, H->wg_per_cu, (i & 1) ? b : a, (i & 1) ? a : b, plan[i], H->cap);
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

sqz_status batch_autotune(BatchHost *H, uint8_t *a, uint8_t *b, hipStream_t st, unsigned *best_out)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_error(SQZ_ERR_HIP, "hipEventCreate failed");
    bool has_xt = false;
    for (const BatchInst &I : H->inst) has_xt |= I.kind >= kBX68 && I.kind <= kBXAny;
    const unsigned weights[] = {2, 3, 4, 6, 8};
    unsigned best = H->wg_per_cu, best_w = H->xt_weight;
    float best_ms = 1e30f;
    sqz_status st2 = SQZ_OK;
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
            st2 = launch_batch(H, w, a, b, H->K, st);  // warm-up
            if (st2 != SQZ_OK) break;
            (void)hipEventRecord(e0, st);
            for (int i = 0; i < 4 && st2 == SQZ_OK; ++i)
                st2 = launch_batch(H, w, (i & 1) ? b : a, (i & 1) ? a : b, H->K, st);
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) {
                st2 = set_error(SQZ_ERR_HIP, "autotune synchronisation failed");
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) {
                best_ms = ms;
                best = w;
                best_w = H->xt_weight;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    H->xt_weight = best_w;
    hipError_t e = upload_costs(H);
    if (st2 == SQZ_OK && e != hipSuccess) st2 = hip_error(e, "batch cost upload");
    if (st2 != SQZ_OK) return st2;
    H->wg_per_cu = best;
    if (H->gexec) {
        (void)hipGraphExecDestroy(H->gexec);
        H->gexec = nullptr;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[H->key] = std::make_pair(best, best_w);
    }
    if (best_out) *best_out = best;
    return SQZ_OK;
}

uint64_t batch_total_bytes(const BatchHost *H) { return H->total_bytes; }
uint64_t batch_offset(const BatchHost *H, int32_t i) { return H->offsets[i]; }
int32_t batch_count(const BatchHost *H) { return (int32_t)H->inst.size(); }
unsigned batch_wg_per_cu(const BatchHost *H) { return H->wg_per_cu; }
int batch_steps_per_launch(const BatchHost *H) { return H->K; }
uint64_t batch_total_cells(const BatchHost *H) { return H->total_cells; }

}  // namespace sqz
