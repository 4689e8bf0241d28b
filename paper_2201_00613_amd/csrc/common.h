// Internal declarations shared by the HIP sources of libsqueeze.
//
// Compact storage is one byte (or one float) per fractal cell, in the
// replica-major order: compact index c has base-k digits beta_1..beta_r
// (beta_mu = digit mu-1, least significant first) and lives at expanded
// coordinate lambda(c) = sum_mu tau(beta_mu) * s^(mu-1) (Section
// "Revisiting lambda").  Every level-m subtree is therefore a contiguous
// range [t*k^m, (t+1)*k^m) of the compact array.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "host_tables.h"
#include "squeeze.h"

namespace sqz {

// Device forms of the invariant division (Div32/Div64 in host_tables.h).
__device__ __forceinline__ uint32_t divq(uint32_t n, const Div32 &D)
{
    uint32_t t = __umulhi(D.m, n);
    return (t + ((n - t) >> D.sh1)) >> D.sh2;
}
__device__ __forceinline__ uint64_t divq(uint64_t n, const Div64 &D)
{
    uint64_t t = __umul64hi(D.m, n);
    return (t + ((n - t) >> D.sh1)) >> D.sh2;
}

// Chunked map tables: MapParams (host_tables.h).

// lambda(c) for c < N (Section "Revisiting lambda"); 32-bit index variant
// for N <= 2^32, 64-bit otherwise.
__device__ __forceinline__ void lam_map32(const MapParams &P, uint32_t c, uint32_t &x, uint32_t &y)
{
    uint32_t px = 0, py = 0, sp = 1;
    for (int i = 0; i + 1 < P.nlam; ++i) {
        uint32_t q = divq(c, P.dklam32);
        uint32_t e = P.lam_lo[c - q * P.klam];
        c = q;
        px += (e & 0xFFFFu) * sp;
        py += (e >> 16) * sp;
        sp *= P.slam;
    }
    if (P.nlam > 0) {
        uint32_t e = P.lam_top[c];
        px += (e & 0xFFFFu) * sp;
        py += (e >> 16) * sp;
    }
    x = px;
    y = py;
}

__device__ __forceinline__ void lam_map64(const MapParams &P, uint64_t c, uint32_t &x, uint32_t &y)
{
    uint32_t px = 0, py = 0, sp = 1;
    for (int i = 0; i + 1 < P.nlam; ++i) {
        uint64_t q = divq(c, P.dklam64);
        uint32_t e = P.lam_lo[(uint32_t)(c - q * P.klam)];
        c = q;
        px += (e & 0xFFFFu) * sp;
        py += (e >> 16) * sp;
        sp *= P.slam;
    }
    if (P.nlam > 0) {
        uint32_t e = P.lam_top[(uint32_t)c];
        px += (e & 0xFFFFu) * sp;
        py += (e >> 16) * sp;
    }
    x = px;
    y = py;
}

// nu(x, y) (Section "Formulation of nu"), scanning chunks from the least
// significant level up; kHole64 for holes and for points outside [0,n)^2.
__device__ __forceinline__ uint64_t nu_map(const MapParams &P, int32_t x, int32_t y)
{
    if ((uint32_t)x >= (uint32_t)P.n || (uint32_t)y >= (uint32_t)P.n) return kHole64;
    uint32_t ux = (uint32_t)x, uy = (uint32_t)y;
    uint64_t c = 0, kp = 1;
    for (int i = 0; i + 1 < P.nnu; ++i) {
        uint32_t qx = divq(ux, P.dsnu), qy = divq(uy, P.dsnu);
        uint32_t e = P.nu_lo[(ux - qx * P.snu) + P.snu * (uy - qy * P.snu)];
        if (e == kNuHole32) return kHole64;
        c += (uint64_t)e * kp;
        kp *= P.knu;
        ux = qx;
        uy = qy;
    }
    if (P.nnu > 0) {
        uint32_t e = P.nu_top[ux + P.snu_top * uy];
        if (e == kNuHole32) return kHole64;
        c += (uint64_t)e * kp;
    }
    return c;
}

// ---------------------------------------------------------------------------
// Seeded starts.  SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output i+1
// of the generator seeded with `seed` is the MurmurHash3 variant-13
// finaliser applied to seed + (i+1) * 0x9E3779B97F4A7C15.  Cells are keyed
// by their expanded coordinate, i = y*n + x, so compact and expanded
// layouts start from identical states.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Launch sizes for `steps` steps with at most K per launch (temporal
// blocking): launches of K steps and one of the remainder.  Every launch swaps
// the two buffers, so the launch count must have the parity of `steps` for the
// result to land where one-step launches would leave it; if it does not, the
// last launch of two or more steps is split into (n - 1) + 1.
inline std::vector<int> plan_launches(int32_t steps, int K)
{
    std::vector<int> plan((size_t)(steps / K), K);
    if (steps % K) plan.push_back(steps % K);
    if ((plan.size() & 1) != (size_t)(steps & 1))
        for (size_t i = plan.size(); i-- > 0;)
            if (plan[i] >= 2) {
                plan[i] -= 1;
                plan.push_back(1);
                break;
            }
    return plan;
}

// Host helpers (api.hip; the HIP-free ones are in host_tables.h)
sqz_status hip_error(hipError_t e, const char *what);
// map tables of `level` (map_tables) uploaded to new device memory *d_mem; P's table pointers set
sqz_status build_map_params(const FractalHost &F, int level, MapParams &P, void **d_mem);

// Kernel launchers (maps.hip)
sqz_status launch_lambda(const MapParams &P, const uint64_t *idx, int64_t count, int32_t *xy,
                         hipStream_t st);
sqz_status launch_nu(const MapParams &P, const int32_t *xy, int64_t count, uint64_t *idx,
                     hipStream_t st);
sqz_status launch_fill_bernoulli(const MapParams &P, uint64_t seed, uint32_t thresh24, int expanded,
                                 uint8_t *out, hipStream_t st);
sqz_status launch_fill_uniform(const MapParams &P, uint64_t seed, float *out, hipStream_t st);
sqz_status launch_life_cell(const MapParams &P, const uint8_t *in, uint8_t *out, hipStream_t st);

// Matrix-core map variants (mfma_maps.hip)
MfmaParams *mfma_prepare(const FractalHost &F);
void mfma_release(FractalHost &F);
sqz_status launch_lambda_mfma(const FractalHost &F, const uint64_t *idx, int64_t count, int32_t *xy, hipStream_t st);
sqz_status launch_nu_mfma(const FractalHost &F, const int32_t *xy, int64_t count, uint64_t *idx, hipStream_t st);
sqz_status launch_life_cell_mfma(const FractalHost &F, const uint8_t *in, uint8_t *out, hipStream_t st);

// Block-level layouts: lambda(omega) on the expanded array, micro-block storage (blocks.hip)
sqz_status blocks_check(const FractalHost &F, int m, int64_t *side);
uint64_t blocks_bytes(const FractalHost &F, int m);
sqz_status launch_life_blocks(const FractalHost &F, int m, bool expanded, const uint8_t *in, uint8_t *out,
                              hipStream_t st);
sqz_status launch_blocks_convert(const FractalHost &F, int m, bool pack, const uint8_t *src, uint8_t *dst,
                                 hipStream_t st);

// Expanded bounding-box baseline (bb.hip)
sqz_status launch_life_bb(const FractalHost &F, const uint8_t *in, uint8_t *out, hipStream_t st);

// Tiled compact stencil (life_tile.hip)
int tile_kind_for(const FractalHost &F);
sqz_status tile_prepare(FractalHost &F);
void tile_release(FractalHost &F);
int32_t tile_level_of(const FractalHost &F);

// Expanded-tile kernels (xtile.hip)
sqz_status xtile_prepare(FractalHost &F);
void xtile_release(FractalHost &F);
int32_t xtile_level_of(const FractalHost &F);
int xtile_steps_per_launch(const FractalHost &F);  // most steps one expanded-tile launch can take (0: none)
sqz_status launch_life_xtile_steps(const FractalHost &F, const uint8_t *in, uint8_t *out, int steps, hipStream_t st);
sqz_status launch_diffuse_xtile_steps(const FractalHost &F, int dtype, float coef, int rounding, uint64_t seed,
                                      uint64_t step, const void *in, void *out, int steps, hipStream_t st);
sqz_status launch_life_xtile(const FractalHost &F, const uint8_t *in, uint8_t *out, hipStream_t st);
sqz_status launch_diffuse(const FractalHost &F, int dtype, float coef, int rounding, uint64_t seed, uint64_t step,
                          const void *in, void *out, int use_tile, hipStream_t st);
sqz_status launch_mass(const FractalHost &F, int dtype, const void *u, double offset, double *work, hipStream_t st);
// the same sum with the partials in the library's static scratch; *result = the sum
sqz_status launch_mass_noalloc(const FractalHost &F, int dtype, const void *u, double offset, double *result,
                               hipStream_t st);
sqz_status launch_bf16_convert(const FractalHost &F, int encode, const float *u, float offset, uint16_t *b,
                               hipStream_t st);
int mass_grid();

// Bit-row expanded tiles (bitbox.hip)
sqz_status bitbox_prepare(FractalHost &F);
void bitbox_release(FractalHost &F);
int bitbox_steps_per_launch(const FractalHost &F);  // 0: none
int32_t bitbox_level_of(const FractalHost &F);
sqz_status launch_life_bitbox(const FractalHost &F, const uint8_t *in, uint8_t *out, int steps, hipStream_t st);

// Batched Life (batch.hip)
struct BatchHost;
sqz_status batch_create(const sqz_fractal *const *fr, int32_t count, BatchHost **out);
void batch_destroy(BatchHost *H);
sqz_status batch_step(const BatchHost *H, const uint8_t *in, uint8_t *out, hipStream_t st);
sqz_status batch_run(BatchHost *H, uint8_t *a, uint8_t *b, int32_t steps, hipStream_t st);
sqz_status batch_autotune(BatchHost *H, uint8_t *a, uint8_t *b, hipStream_t st, unsigned *best_out);
sqz_status batch_set_tiled(BatchHost *H, int32_t persistent, int32_t steps_per_launch, int32_t wg_per_cu);
uint64_t batch_total_bytes(const BatchHost *H);
uint64_t batch_offset(const BatchHost *H, int32_t i);
int32_t batch_count(const BatchHost *H);
unsigned batch_wg_per_cu(const BatchHost *H);
int batch_steps_per_launch(const BatchHost *H);
void batch_tiled_form(const BatchHost *H, int32_t *form, int32_t *steps_per_launch, int32_t *wg_per_cu);
uint64_t batch_total_cells(const BatchHost *H);
const FractalHost &fractal_host_of(const sqz_fractal *f);
sqz_status launch_life_tile(const FractalHost &F, const uint8_t *in, uint8_t *out, hipStream_t st);
int tile_steps_per_launch(const FractalHost &F);  // most Life steps one tiled launch can take (0: no tiles)
sqz_status launch_life_tile_steps(const FractalHost &F, const uint8_t *in, uint8_t *out, int steps, hipStream_t st);
bool tile_resident(const FractalHost &F);  // the resident run is available
// all steps in one launch with the tiles held in LDS (all on the chip at once); result in a (steps even) or b
sqz_status launch_life_tile_resident(const FractalHost &F, uint8_t *a, uint8_t *b, int steps, hipStream_t st);

}  // namespace sqz
