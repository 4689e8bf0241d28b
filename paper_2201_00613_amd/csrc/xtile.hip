// Expanded-tile kernels (device code in xtile_device.h) and their host side:
// tile level choice, tile-invariant tables, launches; thread-level
// diffusion, binary64 mass and bfloat16 conversion kernels.
#include <string.h>

#include <mutex>
#include <vector>

#include "xtile_device.h"

namespace sqz {

namespace {

template <class Op, int PT>
__global__ void __launch_bounds__(kXBlock) __attribute__((amdgpu_waves_per_eu(Op::kWaves)))
k_xtile(XArgs A, const typename Op::G *__restrict__ in,
                                                   typename Op::G *__restrict__ out, XOp op)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const XLds<Op> S(smem, A);
    xtile_setup<Op>(A, S);
    const uint64_t chunk = (A.ntiles + gridDim.x - 1) / gridDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t t1 = t0 + chunk < A.ntiles ? t0 + chunk : A.ntiles;
    if (A.KM == 16 * 256 && A.R <= 2 * 256)
        xtile_run<Op, PT, 16, 2, true>(A, in, out, t0, t1, op, S);
    else if (A.KM <= 16 * 256 && A.R <= 2 * 256)
        xtile_run<Op, PT, 16, 2>(A, in, out, t0, t1, op, S);
    else
        for (uint64_t t = t0; t < t1; ++t) xtile_body<Op, PT>(A, in, out, t, op, S);
}

// K steps per launch (multi-step expanded tiles).
template <class Op, int PT, int K>
__global__ void __launch_bounds__(kXBlock) k_xtileK(XArgs A, const typename Op::G *__restrict__ in,
                                                    typename Op::G *__restrict__ out, XOp op)
{
    extern __shared__ __align__(16) unsigned char smem[];
    xtile_setupK<Op>(A, smem);
    const uint64_t chunk = (A.ntiles + gridDim.x - 1) / gridDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t t1 = t0 + chunk < A.ntiles ? t0 + chunk : A.ntiles;
    xtile_runK<Op, PT, 16, 4, K>(A, in, out, t0, t1, op, smem);
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

// Folds the kMassGrid partials part[0..kMassGrid) into *result.
__global__ void __launch_bounds__(256) k_mass_final(const double *part, double *result, uint64_t N, double offset)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < kMassGrid; i += 256) acc += part[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) *result = s + (double)N * offset;
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

static sqz_status xtile_prepare_multi(FractalHost &F, XTileConfig *X);

sqz_status xtile_prepare(FractalHost &F)
{
    F.xtile = nullptr;
    if (F.r < 1) return SQZ_OK;
    // the largest level whose expanded tile fits the LDS budget in binary32
    int M = F.r < 12 ? F.r : 12;
    std::vector<XRingSlot> ring;
    for (; M >= 1; --M) {
        uint64_t B = 1, KM = 1;
        for (int i = 0; i < M; ++i) {
            B *= F.s;
            KM *= F.k;
        }
        const uint64_t P = (B + 2 + 3) / 4 * 4;  // ring on both sides, pitch a multiple of 4
        if (P * P > 65535 || KM > 65535) continue;
        if (xt_layout((uint32_t)P, (uint32_t)KM, 0, 4, true, false, nullptr) > kXLdsBudget) continue;
        xtile_ring_slots(F, M, (uint32_t)P, ring);
        if (xt_layout((uint32_t)P, (uint32_t)KM, (uint32_t)ring.size(), 4, true, false, nullptr) <= kXLdsBudget) break;
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
    X->P = (X->B + 2 + 3) / 4 * 4;
    X->R = (uint32_t)ring.size();
    const uint32_t P = X->P, KM = X->KM, R = X->R;

    // tables: lambda positions, cell entries (diffusion), ring positions, ring info
    std::vector<uint16_t> lam;
    std::vector<uint32_t> ent;
    int shifts[8];
    for (int d8 = 0; d8 < 8; ++d8) shifts[d8] = deg_field(d8);
    xtile_cell_entries(F, M, P, shifts, lam, ent);
    const size_t o_lam = 0, o_ent = xt_align16(o_lam + KM * 2), o_rpos = xt_align16(o_ent + (size_t)KM * 4),
                 o_rinfo = xt_align16(o_rpos + (size_t)R * 2), total = xt_align16(o_rinfo + (size_t)R * 4 + 4);
    std::vector<uint8_t> blob(total, 0);
    memcpy(blob.data() + o_lam, lam.data(), KM * 2);
    memcpy(blob.data() + o_ent, ent.data(), (size_t)KM * 4);
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
    X->base.B = X->B;
    X->base.R = R;
    X->base.lam = (const uint16_t *)(b + o_lam);
    X->base.ent = (const uint32_t *)(b + o_ent);
    X->base.rpos = (const uint16_t *)(b + o_rpos);
    X->base.rinfo = (const uint32_t *)(b + o_rinfo);
    X->lds_life = xt_layout(P, KM, R, 1, false, true, nullptr);
    X->lds_diff = xt_layout(P, KM, R, 4, true, false, nullptr);
    X->grid_life = occupancy_grid<XLife, 0>(X->lds_life, X->ntiles, F.device);
    X->grid_diff = occupancy_grid<XDiffF32, 0>(X->lds_diff, X->ntiles, F.device);
    X->grid_diff16 = occupancy_grid<XDiffBF16, 0>(X->lds_diff, X->ntiles, F.device);
    st = xtile_prepare_multi(F, X);
    if (st != SQZ_OK) {
        (void)hipFree(X->d_tab);
        (void)hipFree(X->d_coarse);
        delete X;
        return st;
    }
    F.xtile = X;
    return SQZ_OK;
}

// Multi-step form of an expanded-tile configuration: the same tile level with a
// border of K cells (K = 3 or 2, the largest whose tables fit the LDS budget).
static constexpr size_t kXLdsBudgetK = 53 * 1024;  // three workgroups per CU

template <class Op, int PT, int K>
static unsigned occupancy_gridK(size_t lds, uint64_t ntiles, int device)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_xtileK<Op, PT, K>, kXBlock, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) cus = prop.multiProcessorCount;
    uint64_t g = (uint64_t)cus * (uint64_t)per_cu;
    if (g > ntiles) g = ntiles;
    return (unsigned)(g < 1 ? 1 : g);
}

static sqz_status xtile_prepare_multi(FractalHost &F, XTileConfig *X)
{
    X->K = 0;
    X->d_tabk = nullptr;
    const int M = X->M;
    const int64_t B = X->B;
    const uint32_t KM = X->KM;
    if (KM > 16 * 256) return SQZ_OK;
    for (int K = 3; K >= 2; --K) {
        if (K > B) continue;
        const uint32_t P = (uint32_t)((B + 2 * K + 3) / 4 * 4), rows = (uint32_t)(B + 2 * K);
        if ((uint64_t)P * rows > 65535) continue;
        // ring slots by layer (member cells of the adjacent tiles within K of the box),
        // box positions and membership of the tile's cells
        std::vector<XRingSlot> ring;
        std::vector<uint32_t> start;
        std::vector<uint16_t> lam;
        std::vector<uint8_t> mem;
        xtile_layer_tables(F, M, K, P, rows, ring, start, lam, mem);
        const uint32_t R = (uint32_t)ring.size();
        if (R > 4 * 256) continue;
        const size_t lds_life = xt_layoutK(P, rows, KM, R, 1, true, nullptr);
        const size_t lds_diff = xt_layoutK(P, rows, KM, R, 4, false, nullptr);
        if (lds_life > kXLdsBudgetK || lds_diff > kXLdsBudgetK) continue;
        const size_t o_lam = 0, o_mem = xt_align16(o_lam + KM * 2), o_rpos = xt_align16(o_mem + (size_t)P * rows),
                     o_rinfo = xt_align16(o_rpos + (size_t)R * 2), total = xt_align16(o_rinfo + (size_t)R * 4 + 4);
        std::vector<uint8_t> blob(total, 0);
        memcpy(blob.data() + o_lam, lam.data(), KM * 2);
        memcpy(blob.data() + o_mem, mem.data(), (size_t)P * rows);
        for (uint32_t j = 0; j < R; ++j) {
            memcpy(blob.data() + o_rpos + 2 * j, &ring[j].pos, 2);
            memcpy(blob.data() + o_rinfo + 4 * j, &ring[j].info, 4);
        }
        hipError_t e = hipMalloc(&X->d_tabk, total);
        if (e == hipSuccess) e = hipMemcpy(X->d_tabk, blob.data(), total, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (X->d_tabk) (void)hipFree(X->d_tabk);
            X->d_tabk = nullptr;
            return hip_error(e, "multi-step expanded-tile tables");
        }
        const uint8_t *b = (const uint8_t *)X->d_tabk;
        XArgs &A = X->kbase;
        A = X->base;
        A.P = P;
        A.rows = rows;
        A.K = (uint32_t)K;
        A.R = R;
        for (int d = 0; d < 4; ++d) A.ring_start[d] = start[d <= K ? d : K];
        A.lam = (const uint16_t *)(b + o_lam);
        A.mem_in = b + o_mem;
        A.rpos = (const uint16_t *)(b + o_rpos);
        A.rinfo = (const uint32_t *)(b + o_rinfo);
        X->ldsk_life = lds_life;
        X->ldsk_diff = lds_diff;
        if (K == 3) {
            X->gridk_life = occupancy_gridK<XLife, 0, 3>(lds_life, X->ntiles, F.device);
            X->gridk_diff = occupancy_gridK<XDiffF32, 0, 3>(lds_diff, X->ntiles, F.device);
        } else {
            X->gridk_life = occupancy_gridK<XLife, 0, 2>(lds_life, X->ntiles, F.device);
            X->gridk_diff = occupancy_gridK<XDiffF32, 0, 2>(lds_diff, X->ntiles, F.device);
        }
        X->K = (uint32_t)K;
        return SQZ_OK;
    }
    return SQZ_OK;
}

void xtile_release(FractalHost &F)
{
    if (!F.xtile) return;
    if (F.xtile->d_tabk) (void)hipFree(F.xtile->d_tabk);
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
    const size_t lds = xt_layout(X->P, X->KM, X->R, sizeof(typename Op::L), Op::kMem, Op::kSwar, &A);
    A.vec = ((X->KM * sizeof(typename Op::G)) % 16 == 0 && !(((uintptr_t)in | (uintptr_t)out) & 15)) ? 1u : 0u;
    const unsigned grid = life ? X->grid_life : (sizeof(typename Op::G) == 4 ? X->grid_diff : X->grid_diff16);
    using G = typename Op::G;
    const G *i = (const G *)in;
    G *o = (G *)out;
    switch (X->P) {
    case 68: hipLaunchKernelGGL((k_xtile<Op, 68>), dim3(grid), dim3(kXBlock), lds, st, A, i, o, op); break;
    case 84: hipLaunchKernelGGL((k_xtile<Op, 84>), dim3(grid), dim3(kXBlock), lds, st, A, i, o, op); break;
    default: hipLaunchKernelGGL((k_xtile<Op, 0>), dim3(grid), dim3(kXBlock), lds, st, A, i, o, op); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "expanded-tile launch");
}

// `steps` (1..K) steps per launch with the multi-step form (1: the one-step kernel).
template <class Op>
static sqz_status launch_xK(const FractalHost &F, const void *in, void *out, const XOp &op, int steps, hipStream_t st)
{
    const XTileConfig *X = F.xtile;
    if (steps == 1) return launch_x<Op>(F, in, out, op, st);
    if (steps < 1 || steps > (int)X->K)
        return set_error(SQZ_ERR_UNSUPPORTED, "%d steps per launch exceed the %u of this fractal's tiles", steps, X->K);
    XArgs A = X->kbase;
    const bool life = !Op::kMem;
    const size_t lds = xt_layoutK(A.P, A.rows, A.KM, A.R, sizeof(typename Op::L), life, &A);
    const unsigned grid = life ? X->gridk_life : X->gridk_diff;
    using G = typename Op::G;
    const G *i = (const G *)in;
    G *o = (G *)out;
    if (steps == 3) {
        if (A.P == 88)
            hipLaunchKernelGGL((k_xtileK<Op, 88, 3>), dim3(grid), dim3(kXBlock), lds, st, A, i, o, op);
        else
            hipLaunchKernelGGL((k_xtileK<Op, 0, 3>), dim3(grid), dim3(kXBlock), lds, st, A, i, o, op);
    } else {
        if (A.P == 88)
            hipLaunchKernelGGL((k_xtileK<Op, 88, 2>), dim3(grid), dim3(kXBlock), lds, st, A, i, o, op);
        else
            hipLaunchKernelGGL((k_xtileK<Op, 0, 2>), dim3(grid), dim3(kXBlock), lds, st, A, i, o, op);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "multi-step expanded-tile launch");
}

int xtile_steps_per_launch(const FractalHost &F) { return F.xtile ? (F.xtile->K > 1 ? (int)F.xtile->K : 1) : 0; }

sqz_status launch_life_xtile_steps(const FractalHost &F, const uint8_t *in, uint8_t *out, int steps, hipStream_t st)
{
    if (!F.xtile) return set_error(SQZ_ERR_UNSUPPORTED, "no expanded tile for this fractal");
    XOp op{};
    return launch_xK<XLife>(F, in, out, op, steps, st);
}

sqz_status launch_diffuse_xtile_steps(const FractalHost &F, int dtype, float coef, int rounding, uint64_t seed,
                                      uint64_t step, const void *in, void *out, int steps, hipStream_t st)
{
    if (!F.xtile) return set_error(SQZ_ERR_UNSUPPORTED, "no expanded tile for this fractal");
    XOp op;
    op.coef = coef;
    op.rounding = (uint32_t)rounding;
    op.seed = seed;
    op.step = step;
    return dtype == SQZ_F32 ? launch_xK<XDiffF32>(F, in, out, op, steps, st)
                            : launch_xK<XDiffBF16>(F, in, out, op, steps, st);
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

// The two mass kernels with the partials at `part` (kMassGrid doubles) and
// the sum written to *result.
static sqz_status mass_launches(const FractalHost &F, int dtype, const void *u, double offset, double *part,
                                double *result, hipStream_t st)
{
    if (dtype == SQZ_F32)
        hipLaunchKernelGGL(k_mass_partial<float>, dim3(kMassGrid), dim3(256), 0, st, (const float *)u, F.N, part);
    else
        hipLaunchKernelGGL(k_mass_partial<uint16_t>, dim3(kMassGrid), dim3(256), 0, st, (const uint16_t *)u, F.N,
                           part);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(256), 0, st, (const double *)part, result, F.N, offset);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "mass launch");
}

sqz_status launch_mass(const FractalHost &F, int dtype, const void *u, double offset, double *work, hipStream_t st)
{
    return mass_launches(F, dtype, u, offset, work + 1, work, st);
}

// Partial sums of the allocation-free mass (sqz_mass_f64_noalloc): kMassGrid
// doubles, whatever the fractal's size.  Each GPU the library runs on holds
// its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: kernels get the address that
// hipGetSymbolAddress returns for the current device, looked up on the first
// call on each device and kept in scratch_dev.
static __device__ __align__(256) double scratch[kMassGrid];

constexpr int kMaxDevices = 64;
static double *scratch_dev[kMaxDevices];
static std::mutex scratch_mu;

sqz_status launch_mass_noalloc(const FractalHost &F, int dtype, const void *u, double offset, double *result,
                               hipStream_t st)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error(SQZ_ERR_UNSUPPORTED, "device %d >= %d", dev, kMaxDevices);
    double *part = nullptr;
    {
        std::lock_guard<std::mutex> lock(scratch_mu);
        if (!scratch_dev[dev]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) return hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
            scratch_dev[dev] = static_cast<double *>(p);
        }
        part = scratch_dev[dev];
    }
    const uintptr_t r = (uintptr_t)result, p0 = (uintptr_t)part;
    if (r < p0 + kMassGrid * sizeof(double) && p0 < r + sizeof(double))
        return set_error(SQZ_ERR_INVALID, "d_out lies in the library's scratch");
    return mass_launches(F, dtype, u, offset, part, result, st);
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
