// Host side of libsqueeze: descriptor validation, map-table construction,
// handle management and argument checking for every entry point.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "common.h"

struct sqz_fractal {
    sqz::FractalHost h;
    size_t device_mem;  // total memory of the device the handle lives on
};

struct sqz_batch {
    sqz::BatchHost *h;
    std::vector<const sqz_fractal *> fractals;
    size_t device_mem;
};

namespace sqz {
const FractalHost &fractal_host_of(const sqz_fractal *f) { return f->h; }
}  // namespace sqz

namespace sqz {

sqz_status hip_error(hipError_t e, const char *what)
{
    return set_error(SQZ_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static uint64_t upow(uint64_t b, int e)
{
    uint64_t p = 1;
    while (e-- > 0) p *= b;
    return p;
}

sqz_status build_map_params(const FractalHost &F, int level, MapParams &P, void **d_mem)
{
    MapTables T;
    map_tables(F, level, P, T);
    const size_t total = T.all.size();
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, total * sizeof(uint32_t));
    if (e != hipSuccess) return set_error(SQZ_ERR_NOMEM, "hipMalloc of map tables: %s", hipGetErrorString(e));
    e = hipMemcpy(mem, T.all.data(), total * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return hip_error(e, "hipMemcpy of map tables");
    }
    const uint32_t *base = (const uint32_t *)mem;
    P.lam_lo = base + T.off[0];
    P.lam_top = base + T.off[1];
    P.nu_lo = base + T.off[2];
    P.nu_top = base + T.off[3];
    *d_mem = mem;
    return SQZ_OK;
}

}  // namespace sqz

using namespace sqz;

static void fill_info(const FractalHost &F, sqz_info *out)
{
    memset(out, 0, sizeof *out);
    out->s = F.s;
    out->k = F.k;
    out->r = F.r;
    out->n = F.n;
    out->cells = F.N;
    out->compact_w = upow(F.k, (F.r + 1) / 2);
    out->compact_h = upow(F.k, F.r / 2);
}

extern "C" {

sqz_status sqz_descriptor_check(int32_t s, int32_t k, const int32_t *offsets_xy, int32_t r, sqz_info *out)
{
    FractalHost *F = new (std::nothrow) FractalHost;
    if (!F) return set_error(SQZ_ERR_NOMEM, "host allocation failed");
    sqz_status st = check_descriptor(s, k, offsets_xy, r, F);
    if (st == SQZ_OK && out) fill_info(*F, out);
    delete F;
    return st;
}

sqz_status sqz_fractal_create(int32_t s, int32_t k, const int32_t *offsets_xy, int32_t r, sqz_fractal **out)
{
    if (!out) return set_error(SQZ_ERR_INVALID, "out is NULL");
    sqz_fractal *f = new (std::nothrow) sqz_fractal;
    if (!f) return set_error(SQZ_ERR_NOMEM, "host allocation failed");
    sqz_status st = check_descriptor(s, k, offsets_xy, r, &f->h);
    if (st != SQZ_OK) {
        delete f;
        return st;
    }
    hipError_t e = hipGetDevice(&f->h.device);
    if (e != hipSuccess) {
        delete f;
        return hip_error(e, "hipGetDevice");
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, f->h.device);
    if (e != hipSuccess) {
        delete f;
        return hip_error(e, "hipGetDeviceProperties");
    }
    f->device_mem = prop.totalGlobalMem;
    st = build_map_params(f->h, r, f->h.P, &f->h.d_tables);
    if (st != SQZ_OK) {
        delete f;
        return st;
    }
    f->h.tile_kind = tile_kind_for(f->h);
    f->h.tile = nullptr;
    f->h.xtile = nullptr;
    f->h.bitbox = nullptr;
    f->h.mfma = mfma_prepare(f->h);  // null when the pattern does not fit int8 digits
    if (f->h.tile_kind) st = tile_prepare(f->h);
    if (st == SQZ_OK) st = xtile_prepare(f->h);
    if (st == SQZ_OK) st = bitbox_prepare(f->h);
    if (st != SQZ_OK) {
        tile_release(f->h);
        xtile_release(f->h);
        bitbox_release(f->h);
        mfma_release(f->h);
        (void)hipFree(f->h.d_tables);
        delete f;
        return st;
    }
    *out = f;
    return SQZ_OK;
}

void sqz_fractal_destroy(sqz_fractal *f)
{
    if (!f) return;
    tile_release(f->h);
    xtile_release(f->h);
    bitbox_release(f->h);
    mfma_release(f->h);
    if (f->h.d_tables) (void)hipFree(f->h.d_tables);
    delete f;
}

sqz_status sqz_fractal_info(const sqz_fractal *f, sqz_info *out)
{
    if (!f || !out) return set_error(SQZ_ERR_INVALID, "NULL argument");
    fill_info(f->h, out);
    out->has_tile = f->h.tile_kind != 0;
    out->tile_level = tile_level_of(f->h);
    out->xtile_level = xtile_level_of(f->h);
    out->bits_level = bitbox_level_of(f->h);
    {
        const int kt = tile_steps_per_launch(f->h), kb = bitbox_steps_per_launch(f->h),
                  kx = xtile_steps_per_launch(f->h);
        const int k = f->h.tile_kind ? kt : (f->h.bitbox ? kb : kx);
        out->run_steps_per_launch = k > 1 ? k : 1;
        out->resident_run = tile_resident(f->h) ? 1 : 0;
    }
    return SQZ_OK;
}

static sqz_status check_handle(const sqz_fractal *f)
{
    if (!f) return set_error(SQZ_ERR_INVALID, "fractal handle is NULL");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev != f->h.device)
        return set_error(SQZ_ERR_INVALID, "current device %d is not the handle's device %d", dev, f->h.device);
    return SQZ_OK;
}

static sqz_status check_map_impl(const sqz_fractal *f, sqz_map_impl impl)
{
    if (impl != SQZ_MAP_SCALAR && impl != SQZ_MAP_MFMA) return set_error(SQZ_ERR_INVALID, "unknown map evaluation %d", (int)impl);
    if (impl == SQZ_MAP_MFMA && !f->h.mfma)
        return set_error(SQZ_ERR_UNSUPPORTED, "matrix-core maps need k <= 127 (k = %d)", f->h.k);
    return SQZ_OK;
}

sqz_status sqz_lambda_map_impl(const sqz_fractal *f, sqz_map_impl impl, const uint64_t *d_idx, int64_t count,
                               int32_t *d_xy, void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if ((st = check_map_impl(f, impl)) != SQZ_OK) return st;
    if (count < 0) return set_error(SQZ_ERR_INVALID, "count < 0");
    if (count == 0) return SQZ_OK;
    if (!d_idx || !d_xy) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (impl == SQZ_MAP_MFMA) return launch_lambda_mfma(f->h, d_idx, count, d_xy, (hipStream_t)stream);
    return launch_lambda(f->h.P, d_idx, count, d_xy, (hipStream_t)stream);
}

sqz_status sqz_nu_map_impl(const sqz_fractal *f, sqz_map_impl impl, const int32_t *d_xy, int64_t count,
                           uint64_t *d_idx, void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if ((st = check_map_impl(f, impl)) != SQZ_OK) return st;
    if (count < 0) return set_error(SQZ_ERR_INVALID, "count < 0");
    if (count == 0) return SQZ_OK;
    if (!d_idx || !d_xy) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (impl == SQZ_MAP_MFMA) return launch_nu_mfma(f->h, d_xy, count, d_idx, (hipStream_t)stream);
    return launch_nu(f->h.P, d_xy, count, d_idx, (hipStream_t)stream);
}

sqz_status sqz_lambda_map(const sqz_fractal *f, const uint64_t *d_idx, int64_t count, int32_t *d_xy, void *stream)
{
    return sqz_lambda_map_impl(f, SQZ_MAP_SCALAR, d_idx, count, d_xy, stream);
}

sqz_status sqz_nu_map(const sqz_fractal *f, const int32_t *d_xy, int64_t count, uint64_t *d_idx, void *stream)
{
    return sqz_nu_map_impl(f, SQZ_MAP_SCALAR, d_xy, count, d_idx, stream);
}

sqz_status sqz_fill_bernoulli(const sqz_fractal *f, uint64_t seed, double p, sqz_layout layout, uint8_t *d_state,
                              void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if (!d_state) return set_error(SQZ_ERR_INVALID, "d_state is NULL");
    if (!(p >= 0.0 && p <= 1.0)) return set_error(SQZ_ERR_INVALID, "p=%g outside [0,1]", p);
    if (layout != SQZ_LAYOUT_COMPACT && layout != SQZ_LAYOUT_EXPANDED)
        return set_error(SQZ_ERR_INVALID, "unknown layout %d", (int)layout);
    if (layout == SQZ_LAYOUT_EXPANDED && (uint64_t)f->h.n * (uint64_t)f->h.n > f->device_mem)
        return set_error(SQZ_ERR_RANGE, "expanded grid of %lld^2 bytes exceeds device memory", (long long)f->h.n);
    uint32_t thresh = (uint32_t)floor(p * 16777216.0);
    return launch_fill_bernoulli(f->h.P, seed, thresh, layout == SQZ_LAYOUT_EXPANDED, d_state, (hipStream_t)stream);
}

sqz_status sqz_fill_uniform(const sqz_fractal *f, uint64_t seed, float *d_u, void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if (!d_u) return set_error(SQZ_ERR_INVALID, "d_u is NULL");
    return launch_fill_uniform(f->h.P, seed, d_u, (hipStream_t)stream);
}

static bool ranges_overlap(const void *a, uint64_t na, const void *b, uint64_t nb)
{
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

static bool overlap(const void *a, const void *b, uint64_t bytes) { return ranges_overlap(a, bytes, b, bytes); }

sqz_status sqz_compact_step_impl(const sqz_fractal *f, sqz_impl impl, const uint8_t *d_in, uint8_t *d_out,
                                 void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if (!d_in || !d_out) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (overlap(d_in, d_out, f->h.N)) return set_error(SQZ_ERR_INVALID, "d_in and d_out overlap");
    hipStream_t s = (hipStream_t)stream;
    const bool aligned = !(((uintptr_t)d_in | (uintptr_t)d_out) & 15);
    const bool aligned8 = !(((uintptr_t)d_in | (uintptr_t)d_out) & 7);
    switch (impl) {
    case SQZ_IMPL_AUTO:
        // the bit-sliced tiled kernel moves 16-byte words, the bit-row tiles 8-byte
        // words; unaligned buffers skip them
        if (f->h.tile_kind && aligned) return launch_life_tile(f->h, d_in, d_out, s);
        if (f->h.bitbox && aligned8) return launch_life_bitbox(f->h, d_in, d_out, 1, s);
        if (f->h.xtile) return launch_life_xtile(f->h, d_in, d_out, s);
        return launch_life_cell(f->h.P, d_in, d_out, s);
    case SQZ_IMPL_BITS:
        return launch_life_bitbox(f->h, d_in, d_out, 1, s);
    case SQZ_IMPL_CELL:
        return launch_life_cell(f->h.P, d_in, d_out, s);
    case SQZ_IMPL_TILE:
        if (!f->h.tile_kind)
            return set_error(SQZ_ERR_UNSUPPORTED, "no bit-sliced tiled kernel for this replica pattern and level");
        return launch_life_tile(f->h, d_in, d_out, s);
    case SQZ_IMPL_XTILE:
        if (!f->h.xtile) return set_error(SQZ_ERR_UNSUPPORTED, "no expanded tile fits this fractal");
        return launch_life_xtile(f->h, d_in, d_out, s);
    case SQZ_IMPL_CELL_MFMA:
        if (!f->h.mfma) return set_error(SQZ_ERR_UNSUPPORTED, "matrix-core maps need k <= 127 (k = %d)", f->h.k);
        return launch_life_cell_mfma(f->h, d_in, d_out, s);
    }
    return set_error(SQZ_ERR_INVALID, "unknown implementation %d", (int)impl);
}

sqz_status sqz_compact_step(const sqz_fractal *f, const uint8_t *d_in, uint8_t *d_out, void *stream)
{
    return sqz_compact_step_impl(f, SQZ_IMPL_AUTO, d_in, d_out, stream);
}

sqz_status sqz_compact_run(const sqz_fractal *f, uint8_t *d_a, uint8_t *d_b, int32_t steps, void *stream)
{
    return sqz_compact_run_form(f, SQZ_RUN_AUTO, d_a, d_b, steps, stream);
}

// SQZ_RUN_AUTO's choice on aligned buffers: the resident run when it is offered
// and either the run is long enough for its fixed cost (loading and storing
// every tile once: at level 16 it is ahead of launches of ten steps from 10
// steps on) or the launches would need a one-step launch of their own to land
// the result in the buffer of the step count's parity.
constexpr int32_t kAutoResidentSteps = 10;

static bool auto_resident(const FractalHost &h, int32_t steps)
{
    if (steps < 2 || !tile_resident(h)) return false;
    if (steps >= kAutoResidentSteps) return true;
    const int K = tile_steps_per_launch(h);
    return plan_launches(steps, K).size() > (size_t)((steps + K - 1) / K);
}

sqz_status sqz_run_form_auto(const sqz_fractal *f, int32_t steps, sqz_run_form *form)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if (!form) return set_error(SQZ_ERR_INVALID, "NULL form");
    if (steps < 0) return set_error(SQZ_ERR_INVALID, "steps < 0");
    *form = auto_resident(f->h, steps) ? SQZ_RUN_RESIDENT : SQZ_RUN_LAUNCHES;
    return SQZ_OK;
}

sqz_status sqz_compact_run_form(const sqz_fractal *f, sqz_run_form form, uint8_t *d_a, uint8_t *d_b, int32_t steps,
                                void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if (form != SQZ_RUN_AUTO && form != SQZ_RUN_LAUNCHES && form != SQZ_RUN_RESIDENT)
        return set_error(SQZ_ERR_INVALID, "unknown run form %d", (int)form);
    if (steps < 0) return set_error(SQZ_ERR_INVALID, "steps < 0");
    if (!d_a || !d_b) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (overlap(d_a, d_b, f->h.N)) return set_error(SQZ_ERR_INVALID, "d_a and d_b overlap");
    const bool aligned = !(((uintptr_t)d_a | (uintptr_t)d_b) & 15);
    if (form == SQZ_RUN_RESIDENT) {
        if (!tile_resident(f->h))
            return set_error(SQZ_ERR_UNSUPPORTED, "no resident run: the tiles of this fractal do not fit the chip at once");
        if (!aligned) return set_error(SQZ_ERR_INVALID, "the resident run needs 16-byte aligned buffers");
        return launch_life_tile_resident(f->h, d_a, d_b, steps, (hipStream_t)stream);
    }
    if (form == SQZ_RUN_AUTO && aligned && auto_resident(f->h, steps))
        return launch_life_tile_resident(f->h, d_a, d_b, steps, (hipStream_t)stream);
    const bool aligned8 = !(((uintptr_t)d_a | (uintptr_t)d_b) & 7);
    const bool tiled = f->h.tile_kind && aligned, bits = !tiled && f->h.bitbox && aligned8;
    const int K = tiled ? tile_steps_per_launch(f->h)
                        : (bits ? bitbox_steps_per_launch(f->h) : xtile_steps_per_launch(f->h));
    if (K >= 2) {
        const std::vector<int> plan = plan_launches(steps, K);
        const hipStream_t s = (hipStream_t)stream;
        for (size_t i = 0; i < plan.size() && st == SQZ_OK; ++i) {
            const uint8_t *in = (i & 1) ? d_b : d_a;
            uint8_t *out = (i & 1) ? d_a : d_b;
            if (tiled)
                st = launch_life_tile_steps(f->h, in, out, plan[i], s);
            else if (bits)
                st = launch_life_bitbox(f->h, in, out, plan[i], s);
            else
                st = launch_life_xtile_steps(f->h, in, out, plan[i], s);
        }
        return st;
    }
    for (int32_t i = 0; i < steps; ++i) {
        const uint8_t *in = (i & 1) ? d_b : d_a;
        uint8_t *out = (i & 1) ? d_a : d_b;
        st = sqz_compact_step_impl(f, SQZ_IMPL_AUTO, in, out, stream);
        if (st != SQZ_OK) return st;
    }
    return SQZ_OK;
}

static sqz_status check_block_buffers(const void *a, const void *b, uint64_t bytes)
{
    if (!a || !b) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (((uintptr_t)a | (uintptr_t)b) & 3) return set_error(SQZ_ERR_INVALID, "buffers must be 4-byte aligned");
    if (overlap(a, b, bytes)) return set_error(SQZ_ERR_INVALID, "buffers overlap");
    return SQZ_OK;
}

sqz_status sqz_lambda_omega_step(const sqz_fractal *f, int32_t block_level, const uint8_t *d_in, uint8_t *d_out,
                                 void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if ((st = blocks_check(f->h, block_level, nullptr)) != SQZ_OK) return st;
    const uint64_t n = (uint64_t)f->h.n;
    if ((st = check_block_buffers(d_in, d_out, n * n)) != SQZ_OK) return st;
    return launch_life_blocks(f->h, block_level, true, d_in, d_out, (hipStream_t)stream);
}

sqz_status sqz_microblock_bytes(const sqz_fractal *f, int32_t block_level, uint64_t *bytes)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if (!bytes) return set_error(SQZ_ERR_INVALID, "bytes is NULL");
    if ((st = blocks_check(f->h, block_level, nullptr)) != SQZ_OK) return st;
    *bytes = blocks_bytes(f->h, block_level);
    return SQZ_OK;
}

sqz_status sqz_microblock_pack(const sqz_fractal *f, int32_t block_level, const uint8_t *d_compact, uint8_t *d_blocks,
                               void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if ((st = blocks_check(f->h, block_level, nullptr)) != SQZ_OK) return st;
    if (!d_compact || !d_blocks) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (ranges_overlap(d_compact, f->h.N, d_blocks, blocks_bytes(f->h, block_level)))
        return set_error(SQZ_ERR_INVALID, "buffers overlap");
    return launch_blocks_convert(f->h, block_level, true, d_compact, d_blocks, (hipStream_t)stream);
}

sqz_status sqz_microblock_unpack(const sqz_fractal *f, int32_t block_level, const uint8_t *d_blocks,
                                 uint8_t *d_compact, void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if ((st = blocks_check(f->h, block_level, nullptr)) != SQZ_OK) return st;
    if (!d_compact || !d_blocks) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (ranges_overlap(d_compact, f->h.N, d_blocks, blocks_bytes(f->h, block_level)))
        return set_error(SQZ_ERR_INVALID, "buffers overlap");
    return launch_blocks_convert(f->h, block_level, false, d_blocks, d_compact, (hipStream_t)stream);
}

sqz_status sqz_microblock_step(const sqz_fractal *f, int32_t block_level, const uint8_t *d_in, uint8_t *d_out,
                               void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if ((st = blocks_check(f->h, block_level, nullptr)) != SQZ_OK) return st;
    if ((st = check_block_buffers(d_in, d_out, blocks_bytes(f->h, block_level))) != SQZ_OK) return st;
    return launch_life_blocks(f->h, block_level, false, d_in, d_out, (hipStream_t)stream);
}

sqz_status sqz_expanded_step(const sqz_fractal *f, const uint8_t *d_in, uint8_t *d_out, void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    uint64_t n = (uint64_t)f->h.n;
    if (2 * n * n > f->device_mem)
        return set_error(SQZ_ERR_RANGE, "two expanded grids of %llu^2 bytes exceed the device's %zu bytes",
                         (unsigned long long)n, f->device_mem);
    if (!d_in || !d_out) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (overlap(d_in, d_out, n * n)) return set_error(SQZ_ERR_INVALID, "d_in and d_out overlap");
    return launch_life_bb(f->h, d_in, d_out, (hipStream_t)stream);
}

static sqz_status check_diffusion(const sqz_fractal *f, const sqz_diffusion *d)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if (!d) return set_error(SQZ_ERR_INVALID, "diffusion parameters are NULL");
    if (d->dtype != SQZ_F32 && d->dtype != SQZ_BF16) return set_error(SQZ_ERR_INVALID, "unknown dtype %d", (int)d->dtype);
    if (d->rounding != SQZ_ROUND_NEAREST_EVEN && d->rounding != SQZ_ROUND_STOCHASTIC)
        return set_error(SQZ_ERR_INVALID, "unknown rounding %d", (int)d->rounding);
    if (!(d->coef >= 0.0f && d->coef <= 0.125f)) return set_error(SQZ_ERR_INVALID, "coef=%g outside [0, 1/8]", d->coef);
    if (d->impl != SQZ_IMPL_AUTO && d->impl != SQZ_IMPL_CELL && d->impl != SQZ_IMPL_XTILE)
        return set_error(SQZ_ERR_INVALID, "diffusion implementation %d is not AUTO, CELL or XTILE", (int)d->impl);
    if (d->impl == SQZ_IMPL_XTILE && !f->h.xtile) return set_error(SQZ_ERR_UNSUPPORTED, "no expanded tile fits this fractal");
    if (d->steps_per_launch < 0) return set_error(SQZ_ERR_INVALID, "steps_per_launch < 0");
    if (d->steps_per_launch > 1 && (d->impl == SQZ_IMPL_CELL || d->steps_per_launch > xtile_steps_per_launch(f->h)))
        return set_error(SQZ_ERR_UNSUPPORTED, "%d diffusion steps per launch need multi-step expanded tiles (%d here)",
                         d->steps_per_launch, d->impl == SQZ_IMPL_CELL ? 1 : xtile_steps_per_launch(f->h));
    return SQZ_OK;
}

static size_t dtype_size(sqz_dtype t) { return t == SQZ_F32 ? 4 : 2; }

sqz_status sqz_diffuse_step(const sqz_fractal *f, const sqz_diffusion *d, uint64_t step, const void *d_in, void *d_out,
                            void *stream)
{
    sqz_status st = check_diffusion(f, d);
    if (st != SQZ_OK) return st;
    if (!d_in || !d_out) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (overlap(d_in, d_out, f->h.N * dtype_size(d->dtype))) return set_error(SQZ_ERR_INVALID, "d_in and d_out overlap");
    return launch_diffuse(f->h, d->dtype, d->coef, d->rounding, d->seed, step, d_in, d_out, d->impl != SQZ_IMPL_CELL,
                          (hipStream_t)stream);
}

sqz_status sqz_diffuse_run(const sqz_fractal *f, const sqz_diffusion *d, uint64_t first_step, int32_t steps, void *d_a,
                           void *d_b, void *stream)
{
    sqz_status st = check_diffusion(f, d);
    if (st != SQZ_OK) return st;
    if (steps < 0) return set_error(SQZ_ERR_INVALID, "steps < 0");
    if (!d_a || !d_b) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (overlap(d_a, d_b, f->h.N * dtype_size(d->dtype))) return set_error(SQZ_ERR_INVALID, "d_a and d_b overlap");
    const int K = d->steps_per_launch;
    if (K >= 2) {
        const std::vector<int> plan = plan_launches(steps, K);
        uint64_t done = 0;
        for (size_t i = 0; i < plan.size() && st == SQZ_OK; ++i) {
            st = launch_diffuse_xtile_steps(f->h, d->dtype, d->coef, d->rounding, d->seed, first_step + done,
                                            (i & 1) ? d_b : d_a, (i & 1) ? d_a : d_b, plan[i], (hipStream_t)stream);
            done += (uint64_t)plan[i];
        }
        return st;
    }
    for (int32_t i = 0; i < steps; ++i) {
        st = launch_diffuse(f->h, d->dtype, d->coef, d->rounding, d->seed, first_step + (uint64_t)i, (i & 1) ? d_b : d_a,
                            (i & 1) ? d_a : d_b, d->impl != SQZ_IMPL_CELL, (hipStream_t)stream);
        if (st != SQZ_OK) return st;
    }
    return SQZ_OK;
}

sqz_status sqz_mass_f64(const sqz_fractal *f, sqz_dtype dtype, const void *d_u, double offset, double *d_work,
                        void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if (dtype != SQZ_F32 && dtype != SQZ_BF16) return set_error(SQZ_ERR_INVALID, "unknown dtype %d", (int)dtype);
    if (!d_u || !d_work) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (ranges_overlap(d_u, f->h.N * dtype_size(dtype), d_work, SQZ_MASS_WORK_DOUBLES * sizeof(double)))
        return set_error(SQZ_ERR_INVALID, "d_u and d_work overlap");
    return launch_mass(f->h, dtype, d_u, offset, d_work, (hipStream_t)stream);
}

sqz_status sqz_mass_f64_noalloc(const sqz_fractal *f, sqz_dtype dtype, const void *d_u, double offset, double *d_out,
                                void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if (dtype != SQZ_F32 && dtype != SQZ_BF16) return set_error(SQZ_ERR_INVALID, "unknown dtype %d", (int)dtype);
    if (!d_u || !d_out) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (ranges_overlap(d_u, f->h.N * dtype_size(dtype), d_out, sizeof(double)))
        return set_error(SQZ_ERR_INVALID, "d_u and d_out overlap");
    return launch_mass_noalloc(f->h, dtype, d_u, offset, d_out, (hipStream_t)stream);
}

sqz_status sqz_bf16_encode(const sqz_fractal *f, const float *d_u, float offset, uint16_t *d_b, void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if (!d_u || !d_b) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (ranges_overlap(d_u, f->h.N * sizeof(float), d_b, f->h.N * sizeof(uint16_t)))
        return set_error(SQZ_ERR_INVALID, "d_u and d_b overlap");
    return launch_bf16_convert(f->h, 1, d_u, offset, d_b, (hipStream_t)stream);
}

sqz_status sqz_bf16_decode(const sqz_fractal *f, const uint16_t *d_b, float offset, float *d_u, void *stream)
{
    sqz_status st = check_handle(f);
    if (st != SQZ_OK) return st;
    if (!d_u || !d_b) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (ranges_overlap(d_u, f->h.N * sizeof(float), d_b, f->h.N * sizeof(uint16_t)))
        return set_error(SQZ_ERR_INVALID, "d_b and d_u overlap");
    return launch_bf16_convert(f->h, 0, d_u, offset, (uint16_t *)d_b, (hipStream_t)stream);
}

sqz_status sqz_batch_create(int32_t count, const sqz_fractal *const *fractals, sqz_batch **out)
{
    if (!out || !fractals) return set_error(SQZ_ERR_INVALID, "NULL argument");
    if (count < 1) return set_error(SQZ_ERR_INVALID, "count=%d < 1", count);
    for (int32_t i = 0; i < count; ++i) {
        sqz_status st = check_handle(fractals[i]);
        if (st != SQZ_OK) return st;
    }
    sqz_batch *b = new (std::nothrow) sqz_batch;
    if (!b) return set_error(SQZ_ERR_NOMEM, "host allocation failed");
    b->fractals.assign(fractals, fractals + count);
    b->device_mem = fractals[0]->device_mem;
    sqz_status st = batch_create(fractals, count, &b->h);
    if (st != SQZ_OK) {
        delete b;
        return st;
    }
    *out = b;
    return SQZ_OK;
}

void sqz_batch_destroy(sqz_batch *b)
{
    if (!b) return;
    batch_destroy(b->h);
    delete b;
}

sqz_status sqz_batch_layout(const sqz_batch *b, uint64_t *offsets, uint64_t *total_cells)
{
    if (!b) return set_error(SQZ_ERR_INVALID, "batch is NULL");
    const int32_t n = batch_count(b->h);
    if (offsets)
        for (int32_t i = 0; i <= n; ++i) offsets[i] = i < n ? batch_offset(b->h, i) : batch_total_bytes(b->h);
    if (total_cells) *total_cells = batch_total_cells(b->h);
    return SQZ_OK;
}

sqz_status sqz_batch_steps_per_launch(const sqz_batch *b, int32_t *steps)
{
    if (!b || !steps) return set_error(SQZ_ERR_INVALID, "NULL argument");
    *steps = batch_steps_per_launch(b->h);
    return SQZ_OK;
}

static sqz_status check_batch_buffers(const sqz_batch *b, const void *x, const void *y)
{
    if (!b) return set_error(SQZ_ERR_INVALID, "batch is NULL");
    sqz_status st = check_handle(b->fractals[0]);
    if (st != SQZ_OK) return st;
    if (!x || !y) return set_error(SQZ_ERR_INVALID, "NULL buffer");
    if (((uintptr_t)x | (uintptr_t)y) & 15) return set_error(SQZ_ERR_INVALID, "batch buffers must be 16-byte aligned");
    if (overlap(x, y, batch_total_bytes(b->h))) return set_error(SQZ_ERR_INVALID, "batch buffers overlap");
    return SQZ_OK;
}

sqz_status sqz_batch_fill_bernoulli(const sqz_batch *b, const uint64_t *seeds, double p, uint8_t *d_state, void *stream)
{
    if (!b || !seeds || !d_state) return set_error(SQZ_ERR_INVALID, "NULL argument");
    if (((uintptr_t)d_state) & 15) return set_error(SQZ_ERR_INVALID, "batch buffer must be 16-byte aligned");
    const int32_t n = batch_count(b->h);
    for (int32_t i = 0; i < n; ++i) {
        sqz_status st = sqz_fill_bernoulli(b->fractals[i], seeds[i], p, SQZ_LAYOUT_COMPACT,
                                           d_state + batch_offset(b->h, i), stream);
        if (st != SQZ_OK) return st;
    }
    return SQZ_OK;
}

sqz_status sqz_batch_step(const sqz_batch *b, const uint8_t *d_in, uint8_t *d_out, void *stream)
{
    sqz_status st = check_batch_buffers(b, d_in, d_out);
    if (st != SQZ_OK) return st;
    return batch_step(b->h, d_in, d_out, (hipStream_t)stream);
}

sqz_status sqz_batch_run(sqz_batch *b, uint8_t *d_a, uint8_t *d_b, int32_t steps, void *stream)
{
    sqz_status st = check_batch_buffers(b, d_a, d_b);
    if (st != SQZ_OK) return st;
    if (steps < 0) return set_error(SQZ_ERR_INVALID, "steps < 0");
    return batch_run(b->h, d_a, d_b, steps, (hipStream_t)stream);
}

sqz_status sqz_batch_set_tiled_launch(sqz_batch *b, int32_t persistent, int32_t steps_per_launch, int32_t wg_per_cu)
{
    if (!b) return set_error(SQZ_ERR_INVALID, "batch is NULL");
    return batch_set_tiled(b->h, persistent, steps_per_launch, wg_per_cu);
}

sqz_status sqz_batch_tiled_launch(const sqz_batch *b, int32_t *form, int32_t *steps_per_launch, int32_t *wg_per_cu)
{
    if (!b) return set_error(SQZ_ERR_INVALID, "batch is NULL");
    int32_t f = 0, k = 0, w = 0;
    batch_tiled_form(b->h, &f, &k, &w);
    if (form) *form = f;
    if (steps_per_launch) *steps_per_launch = k;
    if (wg_per_cu) *wg_per_cu = w;
    return SQZ_OK;
}

sqz_status sqz_batch_autotune(sqz_batch *b, uint8_t *d_a, uint8_t *d_b, void *stream, int32_t *wg_per_cu)
{
    sqz_status st = check_batch_buffers(b, d_a, d_b);
    if (st != SQZ_OK) return st;
    unsigned best = 0;
    st = batch_autotune(b->h, d_a, d_b, (hipStream_t)stream, &best);
    if (st == SQZ_OK && wg_per_cu) *wg_per_cu = (int32_t)best;
    return st;
}

const char *sqz_status_string(sqz_status st)
{
    switch (st) {
    case SQZ_OK: return "ok";
    case SQZ_ERR_INVALID: return "invalid argument";
    case SQZ_ERR_RANGE: return "size out of range";
    case SQZ_ERR_NOMEM: return "out of memory";
    case SQZ_ERR_HIP: return "HIP runtime error";
    case SQZ_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *sqz_last_error(void) { return last_error_text(); }

}  // extern "C"
