/*
 * squeeze.h -- C ABI of libsqueeze, a compact-fractal stencil library for
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Quezada, Navarro, Hitschfeld, Bustos, "Squeeze: Efficient Compact
 * Fractals for Tensor Core GPUs" (arXiv 2201.00613).  A fractal of the
 * Non-overlapping-Bounding-Boxes (NBB) class is stored in compact form, one
 * value per fractal cell, and neighbourhood computations run on that form
 * through two maps: lambda (compact -> expanded) and nu (expanded ->
 * compact).  The n x n expanded bounding box is never materialised, except
 * by the bounding-box baseline sqz_expanded_step.
 *
 * Conventions for every call:
 *   - Pointers named d_* are device pointers owned by the caller (for
 *     example torch tensors); the library never frees them.  Host pointers
 *     are read before the call returns.
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *     Kernel work is enqueued asynchronously on that stream.
 *   - Argument errors are detected on the host before anything is launched
 *     and leave outputs untouched.  A failed launch returns SQZ_ERR_HIP; a
 *     fault inside a kernel surfaces at the next synchronisation of the
 *     stream (or as SQZ_ERR_HIP from a later call).
 *   - sqz_last_error() returns a message for the calling thread's last
 *     failure.  No C++ exception crosses this interface.
 *
 * Compact layout: the cell with compact index c (0 <= c < N = k^r) has
 * base-k digits beta_1 (least significant) .. beta_r and sits at expanded
 * coordinate lambda(c) = sum_mu tau(beta_mu) s^(mu-1) (Section "Revisiting
 * lambda").  Each level-m subtree is the contiguous range [t k^m, (t+1) k^m).
 * Expanded layout: n x n row-major, byte (x, y) at y*n + x, origin top-left,
 * x to the right, y downwards (Section "Formulation of nu").
 */
#ifndef SQUEEZE_H
#define SQUEEZE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Symbols of the library's public interface (everything else is hidden). */
#if defined(__GNUC__)
#define SQZ_API __attribute__((visibility("default")))
#else
#define SQZ_API
#endif

typedef enum sqz_status {
    SQZ_OK = 0,
    SQZ_ERR_INVALID = 1,     /* malformed argument or descriptor */
    SQZ_ERR_RANGE = 2,       /* sizes overflow the index types or the device */
    SQZ_ERR_NOMEM = 3,       /* a device allocation of the library failed */
    SQZ_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed */
    SQZ_ERR_UNSUPPORTED = 5  /* valid request with no implementation here */
} sqz_status;

/* nu's result for a point that is not a fractal cell (hole or outside the box). */
#define SQZ_HOLE UINT64_MAX

typedef enum sqz_layout { SQZ_LAYOUT_COMPACT = 0, SQZ_LAYOUT_EXPANDED = 1 } sqz_layout;

/* Implementation of the compact stencil.
 *   SQZ_IMPL_AUTO: TILE when the pattern has a bit-sliced tiled kernel and the
 *                  buffers are 16-byte aligned, else BITS when it has bit-row
 *                  tiles and the buffers are 8-byte aligned, else XTILE, else CELL.
 *   SQZ_IMPL_CELL: thread-level Squeeze: one lambda and eight nu per cell
 *                  (Section "Exploring Compact Fractal Space").
 *   SQZ_IMPL_TILE: block-level Squeeze (Section "Moving from Thread-level to
 *                  Block-level"): one coarse map set per level-M subtree, the
 *                  subtree staged on chip.  SQZ_ERR_UNSUPPORTED if the pattern
 *                  has no tiled kernel. */
/*   SQZ_IMPL_XTILE: block-level Squeeze with the level-M subtree expanded on chip
 *                  (any replica pattern; SQZ_ERR_UNSUPPORTED when no level fits).
 *   SQZ_IMPL_CELL_MFMA: CELL with both maps evaluated on the matrix cores
 *                  (SQZ_MAP_MFMA below).  A comparison variant, never chosen by AUTO.
 *   SQZ_IMPL_BITS: block-level Squeeze with the level-M subtree (3 <= M <= 5)
 *                  and a twelve-cell border from the adjacent subtrees expanded
 *                  on chip as bit rows, Life on 32 positions per word (patterns
 *                  with s = 3 and at most 8 replicas that have a kernel: the
 *                  Sierpinski carpet; levels >= 3).  Buffers 8-byte aligned
 *                  (SQZ_ERR_INVALID otherwise); SQZ_ERR_UNSUPPORTED for other
 *                  patterns and levels.  Up to 10 steps per launch in
 *                  sqz_compact_run. */
typedef enum sqz_impl {
    SQZ_IMPL_AUTO = 0,
    SQZ_IMPL_CELL = 1,
    SQZ_IMPL_TILE = 2,
    SQZ_IMPL_XTILE = 3,
    SQZ_IMPL_CELL_MFMA = 4,
    SQZ_IMPL_BITS = 5
} sqz_impl;

/* Evaluation of lambda and nu.
 *   SQZ_MAP_SCALAR: integer arithmetic with chunked look-up tables (several
 *                   levels per table entry).
 *   SQZ_MAP_MFMA: the weighted digit sums as int8 matrix products (the
 *                 encoding of Section "Accelerating Squeeze with Tensor Core
 *                 Units", laid out for v_mfma_i32_32x32x16_i8: 7-bit limbs of
 *                 the level weights times one digit per level, int32
 *                 accumulation).  Exact: a column sum is at most
 *                 r * 127 * (k - 1) < 2^19.  Requires k <= 127
 *                 (SQZ_ERR_UNSUPPORTED otherwise).  Results equal SCALAR's. */
typedef enum sqz_map_impl { SQZ_MAP_SCALAR = 0, SQZ_MAP_MFMA = 1 } sqz_map_impl;

/* How sqz_compact_run_form advances a run.
 *   SQZ_RUN_AUTO: RESIDENT when the fractal offers it (sqz_info.resident_run),
 *                 the buffers are 16-byte aligned, and either steps >= 10 or
 *                 LAUNCHES would need an extra launch to leave the result in the
 *                 buffer the step count's parity names (steps >= 2); else
 *                 LAUNCHES.  The resident run's fixed cost (loading and storing
 *                 every subtree once) pays from about 10 steps, measured on an
 *                 MI355X; sqz_run_form_auto reports the choice.
 *   SQZ_RUN_LAUNCHES: one kernel launch per group of up to
 *                 sqz_info.run_steps_per_launch steps, each reading its input
 *                 buffer whole and writing its output buffer whole (temporal
 *                 blocking within a launch, Section "Moving from Thread-level
 *                 to Block-level" for the tiles).
 *   SQZ_RUN_RESIDENT: all steps in one launch, one workgroup per
 *                 level-M subtree and every subtree held in on-chip memory for
 *                 the whole run; every run_steps_per_launch steps the subtrees
 *                 exchange only the cells their neighbours read (through the
 *                 two caller buffers) at a grid-wide barrier.  Offered for
 *                 patterns with a bit-sliced tiled kernel whose subtrees all fit
 *                 on the chip at once (the level-16 triangle: 729 subtrees of
 *                 level 10).  Runs on one fractal must not overlap on the device
 *                 (each run uses the fractal's barrier counter) and need the
 *                 whole GPU: a run that overlaps another resident run, or
 *                 cannot get all its workgroups on the chip, gives up its
 *                 barrier waits after seconds; the next run call on the
 *                 fractal then returns SQZ_ERR_HIP. */
typedef enum sqz_run_form { SQZ_RUN_AUTO = 0, SQZ_RUN_LAUNCHES = 1, SQZ_RUN_RESIDENT = 2 } sqz_run_form;

/* Storage type of the diffusion field. */
typedef enum sqz_dtype { SQZ_F32 = 0, SQZ_BF16 = 1 } sqz_dtype;

/* Rounding of a binary32 result to bfloat16 storage. */
typedef enum sqz_rounding { SQZ_ROUND_NEAREST_EVEN = 0, SQZ_ROUND_STOCHASTIC = 1 } sqz_rounding;

/* Doubles of caller-provided workspace for sqz_mass_f64 (result in element 0). */
#define SQZ_MASS_WORK_DOUBLES 1025

/* Explicit diffusion on the fractal:
 *   u'_p = u_p + coef * sum over member Moore neighbours q of (u_q - u_p),
 * no flux through holes or the box edge; binary32 arithmetic in a fixed order.
 * SQZ_BF16 storage holds delta = u - offset as bfloat16 (the caller keeps the
 * offset, normally the mean, which the update conserves); the update runs on
 * delta, accumulates in binary32 and rounds per `rounding`, stochastic rounding
 * drawing 16 bits from a counter hash of (seed, step, cell). */
typedef struct sqz_diffusion {
    sqz_dtype dtype;
    sqz_rounding rounding;  /* bfloat16 only */
    float coef;             /* a = dt * alpha; the update is stable for coef <= 1/8 */
    sqz_impl impl;          /* AUTO (= XTILE when available) / CELL / XTILE */
    uint64_t seed;
    int32_t steps_per_launch; /* sqz_diffuse_run with expanded tiles: 0 or 1 = one step per
                                 launch (the default; the update is LDS-bound, so more steps
                                 per launch are slower), 2..3 = that many steps per launch with
                                 multi-step tiles (same results bit for bit); larger values
                                 than the fractal's tiles allow: SQZ_ERR_UNSUPPORTED */
    int32_t reserved;
} sqz_diffusion;

typedef struct sqz_fractal sqz_fractal;

typedef struct sqz_info {
    int32_t s;           /* linear scale factor per level */
    int32_t k;           /* number of replicas */
    int32_t r;           /* level */
    int32_t tile_level;  /* level M of the subtrees the tiled kernel stages (0 if none) */
    int64_t n;           /* side of the expanded box, s^r */
    uint64_t cells;      /* N = k^r, the volume V of Eq. V */
    uint64_t compact_w;  /* width of the paper's compact rectangle, k^ceil(r/2) */
    uint64_t compact_h;  /* height, k^floor(r/2) (Section "Compacting NBB Fractals") */
    int32_t has_tile;    /* 1 if SQZ_IMPL_TILE is available for this pattern */
    int32_t xtile_level; /* level of the expanded tiles of SQZ_IMPL_XTILE (0 if none) */
    int32_t run_steps_per_launch; /* Life steps per launch in sqz_compact_run with aligned buffers:
                                     up to 10 with multi-step tiled kernels (temporal blocking;
                                     16-byte alignment) or bit-row tiles (8-byte), 3 with
                                     multi-step expanded tiles, else 1 */
    int32_t bits_level;  /* level M of the bit-row tiles of SQZ_IMPL_BITS (0 if none) */
    int32_t resident_run; /* 1 if sqz_compact_run_form offers SQZ_RUN_RESIDENT for this fractal */
} sqz_info;

/*
 * Validate an NBB descriptor without touching any device (Introduction:
 * NBB properties; Section "Overview of Squeeze": F_n^{k,s}, r = log_s n).
 *   s: 2..16.  k: 1..s*s.  offsets_xy: k pairs (x, y), replica j is pair j,
 *   each coordinate in [0, s), pairs distinct.  r >= 0 with n = s^r < 2^31
 *   and N = k^r < 2^62.
 * Returns SQZ_ERR_INVALID for a malformed descriptor, SQZ_ERR_RANGE when n
 * or N overflow.  On success fills *out (if not NULL); tile fields are 0.
 */
SQZ_API sqz_status sqz_descriptor_check(int32_t s, int32_t k, const int32_t *offsets_xy, int32_t r,
                                sqz_info *out);

/*
 * Create a fractal handle on the current HIP device: validates as above,
 * builds the map tables on the host and uploads them (synchronously).  The
 * handle owns those device tables; it is immutable and may be used from
 * several threads and streams afterwards.  *out is written only on success.
 * Errors: as sqz_descriptor_check, SQZ_ERR_NOMEM, SQZ_ERR_HIP.
 */
SQZ_API sqz_status sqz_fractal_create(int32_t s, int32_t k, const int32_t *offsets_xy, int32_t r,
                              sqz_fractal **out);

/* Release a handle (NULL is allowed).  Work queued with it must have finished. */
SQZ_API void sqz_fractal_destroy(sqz_fractal *f);

/* Describe a handle. SQZ_ERR_INVALID on NULL arguments. */
SQZ_API sqz_status sqz_fractal_info(const sqz_fractal *f, sqz_info *out);

/*
 * lambda (Section "Revisiting lambda"): compact index -> expanded coordinate.
 *   d_idx: count uint64 compact indices.  d_xy: 2*count int32, (x, y) pairs.
 *   An index >= N yields (-1, -1).  count == 0 is a no-op; count < 0 or a
 *   NULL pointer with count > 0 is SQZ_ERR_INVALID.
 */
SQZ_API sqz_status sqz_lambda_map(const sqz_fractal *f, const uint64_t *d_idx, int64_t count,
                          int32_t *d_xy, void *stream);

/*
 * nu (Section "Formulation of nu"): expanded coordinate -> compact index.
 *   d_xy: 2*count int32 (x, y) pairs.  d_idx: count uint64 results; a point
 *   that is a hole or lies outside [0, n)^2 (negative included) yields
 *   SQZ_HOLE.  Errors as sqz_lambda_map.
 */
SQZ_API sqz_status sqz_nu_map(const sqz_fractal *f, const int32_t *d_xy, int64_t count, uint64_t *d_idx,
                      void *stream);

/* sqz_lambda_map / sqz_nu_map with an explicit evaluation (sqz_map_impl);
 * SQZ_ERR_INVALID for an unknown value. */
SQZ_API sqz_status sqz_lambda_map_impl(const sqz_fractal *f, sqz_map_impl impl, const uint64_t *d_idx,
                                       int64_t count, int32_t *d_xy, void *stream);
SQZ_API sqz_status sqz_nu_map_impl(const sqz_fractal *f, sqz_map_impl impl, const int32_t *d_xy, int64_t count,
                                   uint64_t *d_idx, void *stream);

/*
 * Seeded Bernoulli(p) start, keyed by the expanded coordinate: the cell at
 * (x, y) is 1 iff the top 24 bits of output number y*n+x+1 of SplitMix64
 * seeded with `seed` are below floor(p * 2^24).
 *   layout COMPACT: d_state holds N bytes.  layout EXPANDED: n*n bytes,
 *   holes set to 0.  p outside [0, 1] is SQZ_ERR_INVALID.
 */
SQZ_API sqz_status sqz_fill_bernoulli(const sqz_fractal *f, uint64_t seed, double p, sqz_layout layout,
                              uint8_t *d_state, void *stream);

/*
 * Seeded U(0,1) start in compact layout for the diffusion workload: cell
 * value = (top 24 bits of the same SplitMix64 output) * 2^-24, stored as
 * float (exact).  d_u holds N floats.
 */
SQZ_API sqz_status sqz_fill_uniform(const sqz_fractal *f, uint64_t seed, float *d_u, void *stream);

/*
 * One synchronous step of Conway's Life (B3/S23) on the fractal, compact in
 * and out (Section "Experimental Setup and Results": Moore neighbourhood in
 * expanded space, holes neither simulated nor counted, no wrap at the box).
 *   d_in, d_out: N bytes each, states 0/1 (other values: undefined result).
 *   The two ranges must not overlap (SQZ_ERR_INVALID).
 * Uses SQZ_IMPL_AUTO.
 */
SQZ_API sqz_status sqz_compact_step(const sqz_fractal *f, const uint8_t *d_in, uint8_t *d_out,
                            void *stream);

/* As sqz_compact_step with an explicit implementation choice. */
SQZ_API sqz_status sqz_compact_step_impl(const sqz_fractal *f, sqz_impl impl, const uint8_t *d_in,
                                 uint8_t *d_out, void *stream);

/*
 * `steps` Life steps ping-ponging between d_a and d_b, starting from d_a.
 * The result is in d_a when steps is even, in d_b when odd.  steps >= 0.
 */
SQZ_API sqz_status sqz_compact_run(const sqz_fractal *f, uint8_t *d_a, uint8_t *d_b, int32_t steps,
                           void *stream);

/*
 * As sqz_compact_run (which is form SQZ_RUN_AUTO) with an explicit run form
 * (sqz_run_form above; Section "Experimental Setup and Results": the Life
 * iterations of the benchmark).  Both buffers are read and written: their
 * contents other than the result are unspecified afterwards.
 *   SQZ_RUN_RESIDENT: SQZ_ERR_UNSUPPORTED if the fractal does not offer it,
 *   SQZ_ERR_INVALID for buffers that are not 16-byte aligned.  Unknown forms:
 *   SQZ_ERR_INVALID.
 */
SQZ_API sqz_status sqz_compact_run_form(const sqz_fractal *f, sqz_run_form form, uint8_t *d_a, uint8_t *d_b,
                                        int32_t steps, void *stream);

/*
 * The run form sqz_compact_run (SQZ_RUN_AUTO) takes for `steps` steps on
 * 16-byte aligned buffers: SQZ_RUN_RESIDENT or SQZ_RUN_LAUNCHES, written to
 * *form.  Touches no device.  NULL handle or form, or steps < 0:
 * SQZ_ERR_INVALID.
 */
SQZ_API sqz_status sqz_run_form_auto(const sqz_fractal *f, int32_t steps, sqz_run_form *form);

/*
 * Bounding-box baseline (Section "Experimental Setup and Results", approach
 * BB): the same Life step on the expanded n x n grid, holes written 0.
 *   d_in, d_out: n*n bytes each, non-overlapping, holes of d_in must be 0.
 *   SQZ_ERR_RANGE when two n*n buffers cannot fit in the device's memory
 *   (for example the level-20 triangle: 2 x 1.1 TB).
 */
SQZ_API sqz_status sqz_expanded_step(const sqz_fractal *f, const uint8_t *d_in, uint8_t *d_out,
                             void *stream);

/*
 * Block-level layouts (Section "Moving from Thread-level to Block-level";
 * the approaches compared in Section "Experimental Setup and Results").
 * block_level m: blocks are the level-m subtrees, side s^m (rho in the
 * paper), k^(r-m) of them.  0 <= m <= r and s^m <= 64, else
 * SQZ_ERR_RANGE (m outside [0, r]) or SQZ_ERR_UNSUPPORTED (side > 64).
 * Buffers of the steps must be 4-byte aligned and must not overlap
 * (SQZ_ERR_INVALID).  All steps compute the same Life rule as
 * sqz_compact_step.
 *
 * lambda(omega) approach: states in the expanded n x n array (row-major,
 * as sqz_expanded_step), workgroups launched over the compact grid of
 * blocks, so only the k^(r-m) member blocks are read and written.  Cells
 * outside member blocks are never written: d_out must hold 0 there (a
 * buffer from sqz_fill_bernoulli(..., SQZ_LAYOUT_EXPANDED) or zeroed).
 */
SQZ_API sqz_status sqz_lambda_omega_step(const sqz_fractal *f, int32_t block_level, const uint8_t *d_in,
                                         uint8_t *d_out, void *stream);

/*
 * Micro-block storage (block-level Squeeze memory): block t (compact order)
 * at byte offset t * s^(2m), holding its s^m x s^m box row-major with holes
 * stored as 0; *bytes = k^(r-m) s^(2m).  pack: compact (N bytes) -> blocks,
 * every block byte written.  unpack: blocks -> compact.  step: one Life step
 * from blocks to blocks.
 */
SQZ_API sqz_status sqz_microblock_bytes(const sqz_fractal *f, int32_t block_level, uint64_t *bytes);
SQZ_API sqz_status sqz_microblock_pack(const sqz_fractal *f, int32_t block_level, const uint8_t *d_compact,
                                       uint8_t *d_blocks, void *stream);
SQZ_API sqz_status sqz_microblock_unpack(const sqz_fractal *f, int32_t block_level, const uint8_t *d_blocks,
                                         uint8_t *d_compact, void *stream);
SQZ_API sqz_status sqz_microblock_step(const sqz_fractal *f, int32_t block_level, const uint8_t *d_in,
                                       uint8_t *d_out, void *stream);

/*
 * One diffusion step (see sqz_diffusion).  d_in, d_out: N values of the
 * storage type, non-overlapping.  `step` feeds stochastic rounding only.
 * coef outside [0, 1/8] or an unknown dtype/rounding/impl: SQZ_ERR_INVALID.
 */
SQZ_API sqz_status sqz_diffuse_step(const sqz_fractal *f, const sqz_diffusion *d, uint64_t step, const void *d_in,
                                    void *d_out, void *stream);

/* `steps` diffusion steps ping-ponging from d_a (steps numbered first_step,
 * first_step+1, ...); the result is in d_a when steps is even, else in d_b. */
SQZ_API sqz_status sqz_diffuse_run(const sqz_fractal *f, const sqz_diffusion *d, uint64_t first_step,
                                   int32_t steps, void *d_a, void *d_b, void *stream);

/*
 * Total mass sum_c (offset + u_c) in binary64 on the device, deterministic
 * (fixed reduction tree).  d_u: N values of `dtype`.  d_work: caller-provided
 * device buffer of SQZ_MASS_WORK_DOUBLES doubles; the sum is written to
 * d_work[0], the rest is scratch.  Calls sharing one d_work must not overlap.
 */
SQZ_API sqz_status sqz_mass_f64(const sqz_fractal *f, sqz_dtype dtype, const void *d_u, double offset,
                                double *d_work, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the sum of
 * sqz_mass_f64, bit-identical to it, with no workspace argument.  Its kMassGrid
 * = 1024 partial sums (8 KiB) live in a static device array of the library,
 * one per GPU, held until the process ends; the call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine).  The scratch size does
 * not depend on N, so no fractal is too large for it.  d_out: one double on
 * the device, receives the sum.  Every call on a GPU shares that GPU's
 * scratch: calls that overlap on one GPU (streams not ordered with each other)
 * race and may return wrong sums.  NULL or overlapping buffers, or an unknown
 * dtype: SQZ_ERR_INVALID.
 */
SQZ_API sqz_status sqz_mass_f64_noalloc(const sqz_fractal *f, sqz_dtype dtype, const void *d_u, double offset,
                                        double *d_out, void *stream);

/* bfloat16 storage conversion: d_b[c] = bf16_nearest_even(d_u[c] - offset).
 * d_u: N floats, d_b: N uint16; NULL or overlapping buffers: SQZ_ERR_INVALID. */
SQZ_API sqz_status sqz_bf16_encode(const sqz_fractal *f, const float *d_u, float offset, uint16_t *d_b,
                                   void *stream);

/* d_u[c] = offset + float(d_b[c]); NULL or overlapping buffers: SQZ_ERR_INVALID. */
SQZ_API sqz_status sqz_bf16_decode(const sqz_fractal *f, const uint16_t *d_b, float offset, float *d_u,
                                   void *stream);

/*
 * Batched Life: `count` independent fractals (handles may repeat and may mix
 * replica patterns and levels) advanced together (the batched form of the
 * method's data-parallel step).  Instances with a tiled kernel run as one
 * launch per pattern group or as one launch over all of them, persistent or
 * with a workgroup per tile (sqz_batch_set_tiled_launch; sqz_batch_autotune
 * times all three); the others
 * (expanded tiles, thread level) share one persistent launch.  The handles
 * must outlive the batch and live on the current device.  Instance i owns
 * bytes [offsets[i], offsets[i] + cells_i) of one state buffer of
 * offsets[count] bytes (sqz_batch_layout); the gaps are padding.  A batch is
 * not thread-safe: calls on one batch must not overlap.
 */
typedef struct sqz_batch sqz_batch;

SQZ_API sqz_status sqz_batch_create(int32_t count, const sqz_fractal *const *fractals, sqz_batch **out);

SQZ_API void sqz_batch_destroy(sqz_batch *b);

/* offsets: count + 1 host entries (may be NULL); total_cells: sum of cells_i (may be NULL). */
SQZ_API sqz_status sqz_batch_layout(const sqz_batch *b, uint64_t *offsets, uint64_t *total_cells);

/* Instance i gets sqz_fill_bernoulli(fractal_i, seeds[i], p, COMPACT).  seeds: host array of count. */
SQZ_API sqz_status sqz_batch_fill_bernoulli(const sqz_batch *b, const uint64_t *seeds, double p, uint8_t *d_state,
                                            void *stream);

/* One step of every instance.  Buffers 16-byte aligned, non-overlapping. */
SQZ_API sqz_status sqz_batch_step(const sqz_batch *b, const uint8_t *d_in, uint8_t *d_out, void *stream);

/* `steps` steps ping-ponging from d_a (result in d_a if steps is even, else d_b).  Each launch form
 * follows its own plan of launches of up to its steps per launch (multi-step tiles), with the
 * parity of `steps`.  For steps >= 2 all launches are captured once into a hipGraph (cached for
 * the same buffers and step count) and replayed. */
SQZ_API sqz_status sqz_batch_run(sqz_batch *b, uint8_t *d_a, uint8_t *d_b, int32_t steps, void *stream);

/* Steps every instance advances per launch of sqz_batch_run at least: the smallest steps per
 * launch over the launch forms in use (1 when some instance has no multi-step tiles). */
SQZ_API sqz_status sqz_batch_steps_per_launch(const sqz_batch *b, int32_t *steps);

/* Launch form of the instances with a tiled kernel (triangle, its mirror image, Vicsek cross:
 * bit-sliced tiles; carpet: bit rows):
 *   persistent = 0: one launch per pattern group, one workgroup per tile (the default);
 *   persistent = 1: one persistent launch over all of them, wg_per_cu workgroups per compute unit,
 *                   each taking an equal share of the tiles' cells;
 *   persistent = 2: one launch over all of them, one workgroup per tile (wg_per_cu unused).
 * steps_per_launch: 0 keeps the current value, else 1 .. the most the instances allow (for
 * groups, capped at each group's most).  wg_per_cu: 0 keeps the current value, else 1 .. the
 * most that are resident.  Other values: SQZ_ERR_INVALID.  Results do not depend on the form. */
SQZ_API sqz_status sqz_batch_set_tiled_launch(sqz_batch *b, int32_t persistent, int32_t steps_per_launch,
                                              int32_t wg_per_cu);

/* The launch form in use for the tiled instances (each output may be NULL): *form 0, 1 or 2 as
 * above (-1: no tiled instances); *steps_per_launch of the single launch (forms 1 and 2);
 * *wg_per_cu of the persistent launch (form 1, else 0). */
SQZ_API sqz_status sqz_batch_tiled_launch(const sqz_batch *b, int32_t *form, int32_t *steps_per_launch,
                                          int32_t *wg_per_cu);

/* Time candidate launch shapes on the given buffers (their contents are advanced by a few steps)
 * and keep the fastest for this batch and for later batches of the same composition in this
 * process: for the tiled instances, steps per launch of each pattern group against one launch
 * over all of them (steps per launch x one workgroup per tile or persistent workgroups per
 * compute unit); for the others, workgroups
 * per compute unit and the expanded-tile cost weight.  *wg_per_cu (may be NULL) receives the
 * workgroups per compute unit of the persistent launch timed for the tiled instances (of the
 * other launch when there are none). */
SQZ_API sqz_status sqz_batch_autotune(sqz_batch *b, uint8_t *d_a, uint8_t *d_b, void *stream, int32_t *wg_per_cu);

/* Static text for a status code. */
SQZ_API const char *sqz_status_string(sqz_status st);

/* Message for the calling thread's most recent failure ("" if none). */
SQZ_API const char *sqz_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SQUEEZE_H */
