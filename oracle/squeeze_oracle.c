/*
 * squeeze_oracle.c -- CPU oracle for the Squeeze compact-fractal stencil.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP library: every function below is
 * written from the paper's definitions in the plainest form available
 * (loops over levels, linear searches, full-grid sweeps), in 64-bit
 * integers and, for the diffusion workload, in IEEE double precision.
 *
 * Paper: F. A. Quezada, C. A. Navarro, N. Hitschfeld, B. Bustos,
 * "Squeeze: Efficient Compact Fractals for Tensor Core GPUs", arXiv 2201.00613.
 *
 * A fractal is given as (s, k, offsets, r): scale factor s, k replica
 * offsets tau_j = (offs[2j], offs[2j+1]) in [0,s)^2, level r.  n = s^r is
 * the side of the expanded bounding box and N = k^r the number of cells.
 * A "HOLE" result (-1) marks a point that is not a fractal cell, including
 * every point outside [0,n)^2.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_HOLE (-1LL)

static int64_t ipow(int64_t b, int e)
{
    int64_t p = 1;
    while (e-- > 0) p *= b;
    return p;
}

int orc_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Fractal construction and the two space maps                         */
/* ------------------------------------------------------------------ */

/*
 * Definition of the NBB class (Introduction) and the volume V = k^r
 * (Section "Overview of Squeeze"): level 0 is a single cell at the origin;
 * level mu is made of k copies of level mu-1, copy j translated by
 * tau_j * s^(mu-1).  The compact order is the concatenation of the copies
 * in replica order, which is the "unrolling" of Section "Compacting NBB
 * Fractals" laid out as one linear array (the paper fixes the compact
 * rectangle's size but no memory layout; this linear order is the reading
 * used throughout).
 * Output: xy[2c], xy[2c+1] = expanded coordinate of compact cell c,
 * for c in [0, k^r).
 */
void orc_build_order(int s, int k, const int32_t *offs, int r, int32_t *xy)
{
    int64_t len = 1, scale = 1;
    xy[0] = 0;
    xy[1] = 0;
    for (int mu = 1; mu <= r; ++mu) {
        /* copy j = k-1 .. 1 first, then shift copy 0 in place */
        for (int j = k - 1; j >= 0; --j)
            for (int64_t i = 0; i < len; ++i) {
                xy[2 * (j * len + i)] = (int32_t)(xy[2 * i] + offs[2 * j] * scale);
                xy[2 * (j * len + i) + 1] = (int32_t)(xy[2 * i + 1] + offs[2 * j + 1] * scale);
            }
        len *= k;
        scale *= s;
    }
}

/*
 * lambda (Section "Revisiting lambda", equations for lambda, Delta_mu, tau):
 * lambda(c) = sum_{mu=1..r} tau(beta_mu) * s^(mu-1), where beta_mu is the
 * level-mu replica index.  For the linear compact index c, beta_mu is the
 * base-k digit mu-1 of c (the paper's beta equation reads the same digits
 * out of its 2-D compact coordinate, alternating axes by level).
 */
void orc_lambda(int s, int k, const int32_t *offs, int r, uint64_t c, int64_t *x, int64_t *y)
{
    int64_t px = 0, py = 0, scale = 1;
    for (int mu = 1; mu <= r; ++mu) {
        int beta = (int)(c % (uint64_t)k);
        c /= (uint64_t)k;
        px += offs[2 * beta] * scale;
        py += offs[2 * beta + 1] * scale;
        scale *= s;
    }
    *x = px;
    *y = py;
}

/*
 * nu (Section "Formulation of nu"): top-down over the levels mu = r..1.
 * At level mu the point's digit pair theta_mu = (floor(x/s^(mu-1)) mod s,
 * floor(y/s^(mu-1)) mod s) names the replica it lies in; H_nu is written
 * out as a linear search of the offset list.  A digit pair that is no
 * replica makes the point a hole.  The replica numbers accumulate with
 * weight k^(mu-1) (the linear-index form of the Delta^nu offsets).
 */
int64_t orc_nu(int s, int k, const int32_t *offs, int r, int64_t x, int64_t y)
{
    int64_t n = ipow(s, r);
    if (x < 0 || y < 0 || x >= n || y >= n) return ORC_HOLE;
    int64_t c = 0;
    for (int mu = r; mu >= 1; --mu) {
        int64_t sc = ipow(s, mu - 1);
        int qx = (int)((x / sc) % s), qy = (int)((y / sc) % s);
        int j = 0;
        while (j < k && !(offs[2 * j] == qx && offs[2 * j + 1] == qy)) ++j;
        if (j == k) return ORC_HOLE;
        c += (int64_t)j * ipow(k, mu - 1);
    }
    return c;
}

void orc_lambda_batch(int s, int k, const int32_t *offs, int r, const uint64_t *c,
                      int64_t count, int64_t *xy)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) orc_lambda(s, k, offs, r, c[i], &xy[2 * i], &xy[2 * i + 1]);
}

void orc_nu_batch(int s, int k, const int32_t *offs, int r, const int64_t *xy, int64_t count,
                  int64_t *c)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) c[i] = orc_nu(s, k, offs, r, xy[2 * i], xy[2 * i + 1]);
}

/* Dense inverse of the compact order over the n x n box: -1 on holes. */
void orc_dense_inverse(int s, int k, int r, const int32_t *xy, int64_t *dense)
{
    int64_t n = ipow(s, r), N = ipow(k, r);
    for (int64_t i = 0; i < n * n; ++i) dense[i] = ORC_HOLE;
    for (int64_t c = 0; c < N; ++c) dense[(int64_t)xy[2 * c + 1] * n + xy[2 * c]] = c;
}

/* ------------------------------------------------------------------ */
/* Initial states                                                      */
/* ------------------------------------------------------------------ */

/*
 * SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014): the state advances by the
 * odd constant 0x9E3779B97F4A7C15 and every output is the state passed
 * through the variant-13 finaliser of MurmurHash3.  Output number i+1 of
 * the generator seeded with `seed` is therefore mix(seed + (i+1)*gamma).
 */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Bernoulli start keyed by the expanded coordinate: alive iff the top 24
   bits of output number y*n+x+1 are below thresh24 = floor(p * 2^24). */
static uint8_t bernoulli_cell(uint64_t seed, uint32_t thresh24, int64_t n, int64_t x, int64_t y)
{
    uint64_t h = orc_splitmix64(seed, (uint64_t)(y * n + x));
    return (uint8_t)((h >> 40) < (uint64_t)thresh24);
}

void orc_fill_compact(int s, int k, const int32_t *offs, int r, uint64_t seed, uint32_t thresh24,
                      uint64_t c0, uint64_t c1, uint8_t *out)
{
    int64_t n = ipow(s, r);
#pragma omp parallel for schedule(static)
    for (int64_t c = (int64_t)c0; c < (int64_t)c1; ++c) {
        int64_t x, y;
        orc_lambda(s, k, offs, r, (uint64_t)c, &x, &y);
        out[c - (int64_t)c0] = bernoulli_cell(seed, thresh24, n, x, y);
    }
}

void orc_fill_expanded(int s, int k, const int32_t *offs, int r, uint64_t seed, uint32_t thresh24,
                       uint8_t *out)
{
    int64_t n = ipow(s, r);
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < n; ++y)
        for (int64_t x = 0; x < n; ++x)
            out[y * n + x] = orc_nu(s, k, offs, r, x, y) == ORC_HOLE
                                 ? 0 : bernoulli_cell(seed, thresh24, n, x, y);
}

/* U(0,1) start for the diffusion workload: top 24 bits of the same output,
   times 2^-24 (exact in binary32 and binary64). */
void orc_fill_uniform_compact(int s, int k, const int32_t *offs, int r, uint64_t seed,
                              uint64_t c0, uint64_t c1, double *out)
{
    int64_t n = ipow(s, r);
#pragma omp parallel for schedule(static)
    for (int64_t c = (int64_t)c0; c < (int64_t)c1; ++c) {
        int64_t x, y;
        orc_lambda(s, k, offs, r, (uint64_t)c, &x, &y);
        uint64_t h = orc_splitmix64(seed, (uint64_t)(y * n + x));
        out[c - (int64_t)c0] = (double)(h >> 40) / 16777216.0;
    }
}

/* ------------------------------------------------------------------ */
/* Game of Life on the fractal                                         */
/* ------------------------------------------------------------------ */

/* Rule B3/S23. */
static uint8_t life_rule(uint8_t self, int cnt) { return (uint8_t)(cnt == 3 || (self && cnt == 2)); }

/*
 * Section "Experimental Setup and Results": Conway's Life on the fractal,
 * Moore neighbourhood taken in expanded space, holes skipped (neither
 * simulated nor counted).  On the expanded n x n grid: a member cell counts
 * its member neighbours inside the box (no wrap); non-members are 0.
 * Returns the number of input bytes that are not 0/1 (precondition).
 */
int64_t orc_life_expanded(int64_t n, const uint8_t *member, const uint8_t *in, uint8_t *out)
{
    int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t y = 0; y < n; ++y)
        for (int64_t x = 0; x < n; ++x) {
            int64_t p = y * n + x;
            if (in[p] > 1) ++bad;
            if (!member[p]) {
                out[p] = 0;
                continue;
            }
            int cnt = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy) continue;
                    int64_t qx = x + dx, qy = y + dy;
                    if (qx < 0 || qy < 0 || qx >= n || qy >= n) continue;
                    int64_t q = qy * n + qx;
                    if (member[q]) cnt += in[q];
                }
            out[p] = life_rule(in[p], cnt);
        }
    return bad;
}

/*
 * The same rule computed the Squeeze way on compact storage (Section
 * "Exploring Compact Fractal Space"): lambda once per cell, then nu for
 * each of the 8 Moore neighbours; a HOLE neighbour is skipped.  Computes
 * cells [c0, c1) into out[0 .. c1-c0).  Returns the count of non-0/1 inputs
 * seen among the cells and neighbours it read.
 */
int64_t orc_life_compact(int s, int k, const int32_t *offs, int r, const uint8_t *in,
                         uint64_t c0, uint64_t c1, uint8_t *out)
{
    int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t c = (int64_t)c0; c < (int64_t)c1; ++c) {
        int64_t x, y;
        orc_lambda(s, k, offs, r, (uint64_t)c, &x, &y);
        int cnt = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy) continue;
                int64_t q = orc_nu(s, k, offs, r, x + dx, y + dy);
                if (q == ORC_HOLE) continue;
                if (in[q] > 1) ++bad;
                cnt += in[q];
            }
        if (in[c] > 1) ++bad;
        out[c - (int64_t)c0] = life_rule(in[c], cnt);
    }
    return bad;
}

/*
 * Light cone: a cell's state after t synchronous steps depends only on the
 * starting states within Chebyshev distance t.  The window of side 2t+1
 * centred on (x,y) is filled from the Bernoulli start (non-members and
 * points outside the box are dead and stay dead), advanced t steps with
 * everything outside the window treated as dead, and the centre is read.
 * Errors from the window's edge move inward one cell per step and cannot
 * reach the centre within t steps.
 */
static uint8_t light_cone_one(int s, int k, const int32_t *offs, int r, uint64_t seed,
                              uint32_t thresh24, int64_t x, int64_t y, int t, uint8_t *mem,
                              uint8_t *cur, uint8_t *nxt)
{
    int64_t n = ipow(s, r);
    int w = 2 * t + 1;
    for (int j = 0; j < w; ++j)
        for (int i = 0; i < w; ++i) {
            int64_t px = x - t + i, py = y - t + j;
            int m = orc_nu(s, k, offs, r, px, py) != ORC_HOLE;
            mem[j * w + i] = (uint8_t)m;
            cur[j * w + i] = m ? bernoulli_cell(seed, thresh24, n, px, py) : 0;
        }
    for (int step = 0; step < t; ++step) {
        for (int j = 0; j < w; ++j)
            for (int i = 0; i < w; ++i) {
                if (!mem[j * w + i]) {
                    nxt[j * w + i] = 0;
                    continue;
                }
                int cnt = 0;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (!dx && !dy) continue;
                        int qi = i + dx, qj = j + dy;
                        if (qi < 0 || qj < 0 || qi >= w || qj >= w) continue;
                        cnt += cur[qj * w + qi];
                    }
                nxt[j * w + i] = life_rule(cur[j * w + i], cnt);
            }
        uint8_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    return cur[t * w + t];
}

void orc_light_cone(int s, int k, const int32_t *offs, int r, uint64_t seed, uint32_t thresh24,
                    const int64_t *xy, int64_t count, int t, uint8_t *out)
{
    int w = 2 * t + 1;
#pragma omp parallel
    {
        uint8_t *buf = (uint8_t *)malloc((size_t)3 * w * w);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < count; ++i)
            out[i] = light_cone_one(s, k, offs, r, seed, thresh24, xy[2 * i], xy[2 * i + 1], t, buf,
                                    buf + w * w, buf + 2 * w * w);
        free(buf);
    }
}

/*
 * The light cone for a whole rectangle at once: the states after t steps of
 * every point of the w x h rectangle with corner (x0, y0) (0 for holes and
 * for points outside the box).  The rectangle grown by t on every side is
 * filled from the Bernoulli start and advanced t steps with everything
 * outside it treated as dead; the error this makes at the grown region's
 * edge moves inward one cell per step, so the rectangle itself is exact.
 * out[j*w + i] is point (x0 + i, y0 + j).
 */
static void life_window_one(int s, int k, const int32_t *offs, int r, uint64_t seed, uint32_t thresh24,
                            int64_t x0, int64_t y0, int w, int h, int t, uint8_t *out)
{
    int64_t n = ipow(s, r);
    int W = w + 2 * t, H = h + 2 * t;
    uint8_t *mem = (uint8_t *)malloc((size_t)W * H);
    uint8_t *cur = (uint8_t *)malloc((size_t)W * H);
    uint8_t *nxt = (uint8_t *)malloc((size_t)W * H);
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            int64_t px = x0 - t + i, py = y0 - t + j;
            int m = orc_nu(s, k, offs, r, px, py) != ORC_HOLE;
            mem[(size_t)j * W + i] = (uint8_t)m;
            cur[(size_t)j * W + i] = m ? bernoulli_cell(seed, thresh24, n, px, py) : 0;
        }
    for (int step = 0; step < t; ++step) {
        for (int j = 0; j < H; ++j)
            for (int i = 0; i < W; ++i) {
                size_t p = (size_t)j * W + i;
                if (!mem[p]) {
                    nxt[p] = 0;
                    continue;
                }
                int cnt = 0;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (!dx && !dy) continue;
                        int qi = i + dx, qj = j + dy;
                        if (qi < 0 || qj < 0 || qi >= W || qj >= H) continue;
                        cnt += cur[(size_t)qj * W + qi];
                    }
                nxt[p] = life_rule(cur[p], cnt);
            }
        uint8_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    for (int j = 0; j < h; ++j)
        for (int i = 0; i < w; ++i) out[(size_t)j * w + i] = cur[(size_t)(j + t) * W + (i + t)];
    free(mem);
    free(cur);
    free(nxt);
}

/* count rectangles of w x h points, corners xy0[2q], xy0[2q+1]; out holds
   count * w * h states, rectangle q at out + q*w*h. */
void orc_life_windows(int s, int k, const int32_t *offs, int r, uint64_t seed, uint32_t thresh24,
                      const int64_t *xy0, int64_t count, int w, int h, int t, uint8_t *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < count; ++q)
        life_window_one(s, k, offs, r, seed, thresh24, xy0[2 * q], xy0[2 * q + 1], w, h, t,
                        out + (size_t)q * w * h);
}

/* ------------------------------------------------------------------ */
/* Explicit diffusion on the fractal, binary64                         */
/* ------------------------------------------------------------------ */

/*
 * The PDE application mentioned in the Introduction, in the form fixed for
 * this project: u'_p = u_p + a * sum_{q in N8(p), q in F} (u_q - u_p), unit
 * weight on all eight Moore neighbours, no flux through holes or the box
 * edge.  lambda once per cell and nu per neighbour, as for the Life rule.
 * Computes cells [c0, c1) into out[0 .. c1-c0).
 */
void orc_diffuse_compact(int s, int k, const int32_t *offs, int r, double a, const double *in,
                         uint64_t c0, uint64_t c1, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = (int64_t)c0; c < (int64_t)c1; ++c) {
        int64_t x, y;
        orc_lambda(s, k, offs, r, (uint64_t)c, &x, &y);
        double acc = 0.0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy) continue;
                int64_t q = orc_nu(s, k, offs, r, x + dx, y + dy);
                if (q != ORC_HOLE) acc += in[q] - in[c];
            }
        out[c - (int64_t)c0] = in[c] + a * acc;
    }
}

/*
 * Light cone of the diffusion update: the value of cell (x,y) after t steps
 * depends only on starting values within Chebyshev distance t.  The window of
 * side 2t+1 around it is filled from the U(0,1) start (non-members absent),
 * advanced t steps with no flux out of the window, and the centre is read;
 * the window edge's error moves inward one cell per step.
 */
static double diffuse_cone_one(int s, int k, const int32_t *offs, int r, uint64_t seed, double a, int64_t x,
                               int64_t y, int t, uint8_t *mem, double *cur, double *nxt)
{
    int64_t n = ipow(s, r);
    int w = 2 * t + 1;
    for (int j = 0; j < w; ++j)
        for (int i = 0; i < w; ++i) {
            int64_t px = x - t + i, py = y - t + j;
            int m = orc_nu(s, k, offs, r, px, py) != ORC_HOLE;
            mem[j * w + i] = (uint8_t)m;
            cur[j * w + i] = m ? (double)(orc_splitmix64(seed, (uint64_t)(py * n + px)) >> 40) / 16777216.0 : 0.0;
        }
    for (int step = 0; step < t; ++step) {
        for (int j = 0; j < w; ++j)
            for (int i = 0; i < w; ++i) {
                if (!mem[j * w + i]) {
                    nxt[j * w + i] = 0.0;
                    continue;
                }
                double acc = 0.0;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (!dx && !dy) continue;
                        int qi = i + dx, qj = j + dy;
                        if (qi < 0 || qj < 0 || qi >= w || qj >= w || !mem[qj * w + qi]) continue;
                        acc += cur[qj * w + qi] - cur[j * w + i];
                    }
                nxt[j * w + i] = cur[j * w + i] + a * acc;
            }
        double *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    return cur[t * w + t];
}

void orc_diffuse_cone(int s, int k, const int32_t *offs, int r, uint64_t seed, double a, const int64_t *xy,
                      int64_t count, int t, double *out)
{
    int w = 2 * t + 1;
#pragma omp parallel
    {
        uint8_t *mem = (uint8_t *)malloc((size_t)w * w);
        double *buf = (double *)malloc((size_t)2 * w * w * sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < count; ++i)
            out[i] = diffuse_cone_one(s, k, offs, r, seed, a, xy[2 * i], xy[2 * i + 1], t, mem, buf, buf + w * w);
        free(mem);
        free(buf);
    }
}

/* Neighbour table for repeated diffusion steps: nb[8c+j] = compact index of
   the j-th Moore neighbour (raster order dy, dx) or -1.  Same maps as above,
   evaluated once. */
void orc_neighbour_table(int s, int k, const int32_t *offs, int r, uint64_t c0, uint64_t c1,
                         int64_t *nb)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = (int64_t)c0; c < (int64_t)c1; ++c) {
        int64_t x, y;
        orc_lambda(s, k, offs, r, (uint64_t)c, &x, &y);
        int j = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy) continue;
                nb[8 * (c - (int64_t)c0) + j++] = orc_nu(s, k, offs, r, x + dx, y + dy);
            }
    }
}

/* Diffusion steps over a neighbour table: nsteps explicit updates,
   ping-ponging between u and tmp; the result is left in u. */
void orc_diffuse_table(int64_t N, const int64_t *nb, double a, int nsteps, double *u, double *tmp)
{
    for (int step = 0; step < nsteps; ++step) {
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < N; ++c) {
            double acc = 0.0;
            for (int j = 0; j < 8; ++j) {
                int64_t q = nb[8 * c + j];
                if (q >= 0) acc += u[q] - u[c];
            }
            tmp[c] = u[c] + a * acc;
        }
        memcpy(u, tmp, (size_t)N * sizeof(double));
    }
}

/* Life steps over the same neighbour table (for multi-step references at
   moderate sizes); result left in u. */
void orc_life_table(int64_t N, const int64_t *nb, int nsteps, uint8_t *u, uint8_t *tmp)
{
    for (int step = 0; step < nsteps; ++step) {
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < N; ++c) {
            int cnt = 0;
            for (int j = 0; j < 8; ++j) {
                int64_t q = nb[8 * c + j];
                if (q >= 0) cnt += u[q];
            }
            tmp[c] = life_rule(u[c], cnt);
        }
        memcpy(u, tmp, (size_t)N);
    }
}
