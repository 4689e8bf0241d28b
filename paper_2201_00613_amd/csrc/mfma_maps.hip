// Matrix-core variants of the two space maps and of the thread-level Life
// step.
//
// lambda and nu are weighted digit sums (Sections "Revisiting lambda" and
// "Formulation of nu"): lambda(c) = sum_mu tau(beta_mu) s^(mu-1) and
// nu(x, y) = sum_mu H_nu[theta_mu] k^(mu-1).  The tensor-core encoding of
// Section "Accelerating Squeeze with Tensor Core Units" puts the level
// weights in one operand of a matrix product and the per-level digits in
// the other.  Here the product is laid out for the CDNA int8 matrix
// instruction v_mfma_i32_32x32x16_i8 (D = A B + C, A 32x16, B 16x32):
//   A: row i = 7-bit limb i of the level weights, column = level;
//   B: row = level, column = one probe (a point or a compact index);
//   D: row i, column p = sum over levels of limb_i(weight) * digit(p).
// Sixteen levels per instruction; a second instruction accumulates levels
// 16..31 when r > 16.  The limbs are recombined in 64-bit integers:
// value(p) = sum_i D[i][p] 128^i.
//
// Exactness bound: a digit is at most k - 1 <= 126 (nu, replica index) or
// s - 1 <= 15 (lambda, tau component) and a limb at most 127, so a column
// sum is at most r * 127 * 126 < 2^19 for r <= 30: the int32 accumulators
// hold every partial sum exactly.  All terms are non-negative and the
// recombined value is the map itself (< 2^63), so the 64-bit sum does not
// wrap either.
//
// Digits: with s = 2 a level's digit pair is a bit pair; eight levels are
// spread to bytes with one multiply per nibble and looked up four at a time
// with v_perm_b32 (the 4-entry H_nu table as the permute source).  Other
// s use invariant division per level and an LDS table.  For lambda the
// base-k digits come from invariant division; tau is looked up with
// v_perm_b32 when k <= 8, else from LDS.
//
// Lane layout (wave of 64, lane l = 32 h + p): B operand and D column p;
// lane half h supplies levels 8h..8h+7 (+16 in the second instruction).
// The two halves' partial recombinations are summed with one xor-32
// exchange, after which both lanes of column p hold the value.
#include <cstring>
#include <new>

#include "common.h"

namespace sqz {

typedef int v16i __attribute__((ext_vector_type(16)));

struct MfmaParams {
    int32_t s, k, r, n;
    uint64_t N;
    int32_t nl_nu, nl_lam;  // 7-bit limbs of the largest nu (N - 1) and lambda component (n - 1)
    int32_t passes;         // matrix instructions per product: 1 (r <= 16) or 2
    int32_t s2;             // s == 2: bit digits, byte-permute look-up
    int32_t ksmall;         // k <= 8: tau by byte permute
    uint32_t hnu2;          // s == 2: byte e = replica of digit pair (e & 1, e >> 1), 0x80 = hole
    uint32_t tx[2], ty[2];  // k <= 8: byte b = tau_x(b) / tau_y(b)
    Div32 ds;               // s
    Div32 dsp[4];           // s^(8G), G = 0..3 (only for 8G < r)
    Div32 dk32;             // k, compact indices below 2^32
    Div32 dkp32[4];
    Div64 dk64;             // k, 64-bit compact indices
    Div64 dkp64[4];
    uint8_t hnu[kMaxS * kMaxS];  // replica byte of digit pair theta_x + s theta_y, 0x80 = hole
    uint8_t taux[kMaxK], tauy[kMaxK];
};

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kHoleByte8 = 0x8080808080808080ull;
constexpr uint64_t kLow7Byte8 = 0x7F7F7F7F7F7F7F7Full;

struct MfmaLds {
    uint8_t hnu[kMaxS * kMaxS];
    uint8_t taux[kMaxK], tauy[kMaxK];
};

__device__ __forceinline__ void load_tables(const MfmaParams &M, MfmaLds &L)
{
    for (int i = threadIdx.x; i < kMaxS * kMaxS; i += kBlock) L.hnu[i] = M.hnu[i];
    for (int i = threadIdx.x; i < kMaxK; i += kBlock) {
        L.taux[i] = M.taux[i];
        L.tauy[i] = M.tauy[i];
    }
    __syncthreads();
}

__device__ __forceinline__ int levels_of(const MfmaParams &M, int G)
{
    const int lv = M.r - 8 * G;
    return lv < 0 ? 0 : (lv > 8 ? 8 : lv);
}

__device__ __forceinline__ uint64_t byte_mask(int lv) { return lv >= 8 ? ~0ull : ((1ull << (8 * lv)) - 1); }

// bits 0..3 of v to bytes 0..3
__device__ __forceinline__ uint32_t spread4(uint32_t v) { return (v * 0x00204081u) & 0x01010101u; }

// A operand: byte j = limb `row` of base^(level0 + j) for levels below r.
__device__ __forceinline__ long weight_operand(int row, int nl, int level0, int r, uint64_t base)
{
    if (row >= nl) return 0;
    uint64_t w = 1;
    for (int i = 0; i < level0 && i < r; ++i) w *= base;
    uint64_t out = 0;
    for (int j = 0; j < 8; ++j) {
        if (level0 + j < r) out |= ((w >> (7 * row)) & 127u) << (8 * j);
        w *= base;
    }
    return (long)out;
}

// Replica digits of levels 8G..8G+7 of the in-box point (ux, uy), one byte
// per level; `hole` is set when a level's digit pair is not a replica.
__device__ __forceinline__ uint64_t nu_digits(const MfmaParams &M, const MfmaLds &L, uint32_t ux, uint32_t uy, int G,
                                              bool &hole)
{
    const int lv = levels_of(M, G);
    if (lv == 0) return 0;
    if (M.s2) {
        const uint32_t bx = (ux >> (8 * G)) & 0xFFu, by = (uy >> (8 * G)) & 0xFFu;
        const uint32_t elo = spread4(bx & 15u) + 2u * spread4(by & 15u);
        const uint32_t ehi = spread4(bx >> 4) + 2u * spread4(by >> 4);
        const uint64_t v = (((uint64_t)__builtin_amdgcn_perm(0u, M.hnu2, ehi) << 32) |
                            __builtin_amdgcn_perm(0u, M.hnu2, elo)) &
                           byte_mask(lv);
        hole = hole || (v & kHoleByte8) != 0;
        return v & kLow7Byte8;
    }
    uint32_t xs = divq(ux, M.dsp[G]), ys = divq(uy, M.dsp[G]);
    uint64_t J = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (j < lv) {
            const uint32_t qx = divq(xs, M.ds), qy = divq(ys, M.ds);
            const uint32_t v = L.hnu[(xs - qx * (uint32_t)M.s) + (uint32_t)M.s * (ys - qy * (uint32_t)M.s)];
            hole = hole || (v & 0x80u);
            J |= (uint64_t)(v & 0x7Fu) << (8 * j);
            xs = qx;
            ys = qy;
        }
    }
    return J;
}

// tau_x and tau_y digits of levels 8G..8G+7 of the compact index c < N.
__device__ __forceinline__ void lam_digits(const MfmaParams &M, const MfmaLds &L, uint64_t c, int G, uint64_t &Jx,
                                           uint64_t &Jy)
{
    Jx = Jy = 0;
    const int lv = levels_of(M, G);
    if (lv == 0) return;
    uint64_t B = 0;  // base-k digits, one byte per level
    if (M.N <= 0x100000000ull) {
        uint32_t cs = divq((uint32_t)c, M.dkp32[G]);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j < lv) {
                const uint32_t q = divq(cs, M.dk32);
                B |= (uint64_t)(cs - q * (uint32_t)M.k) << (8 * j);
                cs = q;
            }
        }
    } else {
        uint64_t cs = divq(c, M.dkp64[G]);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j < lv) {
                const uint64_t q = divq(cs, M.dk64);
                B |= (cs - q * (uint64_t)M.k) << (8 * j);
                cs = q;
            }
        }
    }
    const uint64_t m = byte_mask(lv);
    if (M.ksmall) {
        const uint32_t lo = (uint32_t)B, hi = (uint32_t)(B >> 32);
        Jx = ((((uint64_t)__builtin_amdgcn_perm(M.tx[1], M.tx[0], hi)) << 32) | __builtin_amdgcn_perm(M.tx[1], M.tx[0], lo)) & m;
        Jy = ((((uint64_t)__builtin_amdgcn_perm(M.ty[1], M.ty[0], hi)) << 32) | __builtin_amdgcn_perm(M.ty[1], M.ty[0], lo)) & m;
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j < lv) {
                const uint32_t b = (uint32_t)(B >> (8 * j)) & 0xFFu;
                Jx |= (uint64_t)L.taux[b] << (8 * j);
                Jy |= (uint64_t)L.tauy[b] << (8 * j);
            }
        }
    }
}

__device__ __forceinline__ v16i mfma(long a, long b, v16i c) { return __builtin_amdgcn_mfma_i32_32x32x16_i8(a, b, c, 0, 0, 0); }

// This lane's share of sum_i D[i][p] 128^i.  Lane half h holds rows
// 8 (e / 4) + 4 h + e % 4 in element e; limbs 0..8 sit in elements 0..4.
template <int NE>
__device__ __forceinline__ uint64_t limb_sum(const v16i &D, int h, int nl)
{
    uint64_t v = 0;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int row = 8 * (e >> 2) + 4 * h + (e & 3);
        if (row < nl) v += (uint64_t)(uint32_t)D[e] << (7 * row);
    }
    return v;
}

__device__ __forceinline__ uint64_t xor32_sum(uint64_t v)
{
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    const uint32_t olo = (uint32_t)__shfl_xor((int)lo, 32), ohi = (uint32_t)__shfl_xor((int)hi, 32);
    return v + (((uint64_t)ohi << 32) | olo);
}

struct Weights {
    long n0, n1, l0, l1;  // nu and lambda operands, levels 8h.. and 16+8h..
};

__device__ __forceinline__ Weights make_weights(const MfmaParams &M, int p, int h)
{
    Weights W;
    W.n0 = weight_operand(p, M.nl_nu, 8 * h, M.r, (uint64_t)M.k);
    W.n1 = weight_operand(p, M.nl_nu, 16 + 8 * h, M.r, (uint64_t)M.k);
    W.l0 = weight_operand(p, M.nl_lam, 8 * h, M.r, (uint64_t)M.s);
    W.l1 = weight_operand(p, M.nl_lam, 16 + 8 * h, M.r, (uint64_t)M.s);
    return W;
}

// lambda of column p's compact index (every lane of the wave calls this).
__device__ __forceinline__ void lam_column(const MfmaParams &M, const MfmaLds &L, const Weights &W, uint64_t c, int h,
                                           uint32_t &x, uint32_t &y)
{
    v16i Dx = {}, Dy = {};
    uint64_t Jx, Jy;
    lam_digits(M, L, c, h, Jx, Jy);
    Dx = mfma(W.l0, (long)Jx, Dx);
    Dy = mfma(W.l0, (long)Jy, Dy);
    if (M.passes > 1) {
        lam_digits(M, L, c, 2 + h, Jx, Jy);
        Dx = mfma(W.l1, (long)Jx, Dx);
        Dy = mfma(W.l1, (long)Jy, Dy);
    }
    x = (uint32_t)xor32_sum(limb_sum<4>(Dx, h, M.nl_lam));
    y = (uint32_t)xor32_sum(limb_sum<4>(Dy, h, M.nl_lam));
}

// nu of column p's point (every lane of the wave calls this); kHole64 for
// holes and points outside the box.
__device__ __forceinline__ uint64_t nu_column(const MfmaParams &M, const MfmaLds &L, const Weights &W, int32_t px,
                                              int32_t py, int p, int h)
{
    bool hole = (uint32_t)px >= (uint32_t)M.n || (uint32_t)py >= (uint32_t)M.n;
    const uint32_t ux = hole ? 0u : (uint32_t)px, uy = hole ? 0u : (uint32_t)py;
    v16i D = {};
    D = mfma(W.n0, (long)nu_digits(M, L, ux, uy, h, hole), D);
    if (M.passes > 1) D = mfma(W.n1, (long)nu_digits(M, L, ux, uy, 2 + h, hole), D);
    const uint64_t v = xor32_sum(limb_sum<5>(D, h, M.nl_nu));
    const uint64_t m = __ballot(hole);
    return (((m >> p) | (m >> (p + 32))) & 1u) ? kHole64 : v;
}

__global__ void __launch_bounds__(kBlock) k_lambda_mfma(MfmaParams M, const uint64_t *__restrict__ idx, int64_t count,
                                                        int32_t *__restrict__ xy)
{
    __shared__ MfmaLds L;
    load_tables(M, L);
    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const Weights W = make_weights(M, p, h);
    const int64_t chunks = (count + 63) / 64;
    for (int64_t w = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); w < chunks;
         w += (int64_t)gridDim.x * (kBlock / 64)) {
        const int64_t base = w * 64;
        int2 res = make_int2(-1, -1);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t i = base + 32 * q + p;
            const uint64_t c = i < count ? idx[i] : 0;
            const bool ok = c < M.N;
            uint32_t x, y;
            lam_column(M, L, W, ok ? c : 0, h, x, y);
            if (q == h && ok) res = make_int2((int)x, (int)y);
        }
        if (base + lane < count) reinterpret_cast<int2 *>(xy)[base + lane] = res;
    }
}

__global__ void __launch_bounds__(kBlock) k_nu_mfma(MfmaParams M, const int32_t *__restrict__ xy, int64_t count,
                                                    uint64_t *__restrict__ idx)
{
    __shared__ MfmaLds L;
    load_tables(M, L);
    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const Weights W = make_weights(M, p, h);
    const int64_t chunks = (count + 63) / 64;
    for (int64_t w = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); w < chunks;
         w += (int64_t)gridDim.x * (kBlock / 64)) {
        const int64_t base = w * 64;
        uint64_t res = kHole64;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t i = base + 32 * q + p;
            const int2 pt = i < count ? reinterpret_cast<const int2 *>(xy)[i] : make_int2(-1, -1);
            const uint64_t v = nu_column(M, L, W, pt.x, pt.y, p, h);
            if (q == h) res = v;
        }
        if (base + lane < count) idx[base + lane] = res;
    }
}

// Thread-level Squeeze Life (one lambda and eight nu per cell) with both maps
// on the matrix cores.  Lane l owns cell base + l; column p of the products
// is cell base + 32 q + p in instruction pair q, so after lambda every lane
// holds its own cell's point (q = h) and its xor-32 partner's (q = 1 - h),
// which is what the nu columns of both halves need.
__global__ void __launch_bounds__(kBlock) k_life_cell_mfma(MfmaParams M, const uint8_t *__restrict__ in,
                                                           uint8_t *__restrict__ out)
{
    __shared__ MfmaLds L;
    load_tables(M, L);
    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const Weights W = make_weights(M, p, h);
    const uint64_t chunks = (M.N + 63) / 64;
    for (uint64_t w = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); w < chunks;
         w += (uint64_t)gridDim.x * (kBlock / 64)) {
        const uint64_t base = w * 64;
        uint32_t X[2], Y[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint64_t c = base + 32 * q + p;
            lam_column(M, L, W, c < M.N ? c : 0, h, X[q], Y[q]);
        }
        const uint64_t c = base + lane;
        const bool mine = c < M.N;
        uint32_t cnt = 0;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            if (j == 4) continue;
            const int dx = j % 3 - 1, dy = j / 3 - 1;
            uint64_t nb = kHole64;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint64_t v = nu_column(M, L, W, (int32_t)X[q] + dx, (int32_t)Y[q] + dy, p, h);
                if (q == h) nb = v;
            }
            if (mine && nb != kHole64) cnt += in[nb];
        }
        if (mine) {
            const uint32_t self = in[c];
            out[c] = (uint8_t)(cnt == 3 || (self && cnt == 2));
        }
    }
}

unsigned grid_for_waves(uint64_t items)
{
    uint64_t g = (items + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    if (g == 0) g = 1;
    return (unsigned)g;
}

uint32_t bits_of(uint64_t v)
{
    uint32_t b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

}  // namespace

MfmaParams *mfma_prepare(const FractalHost &F)
{
    if (F.k > 127 || F.r > 32) return nullptr;  // digits must fit int8; 32 levels per product
    MfmaParams *M = new (std::nothrow) MfmaParams;
    if (!M) return nullptr;
    memset(M, 0, sizeof(*M));
    M->s = F.s;
    M->k = F.k;
    M->r = F.r;
    M->n = (int32_t)F.n;
    M->N = F.N;
    M->nl_nu = (int32_t)((bits_of(F.N - 1) + 6) / 7);
    M->nl_lam = (int32_t)((bits_of((uint64_t)F.n - 1) + 6) / 7);
    M->passes = F.r > 16 ? 2 : 1;
    M->s2 = F.s == 2;
    M->ksmall = F.k <= 8;
    for (int e = 0; e < F.s * F.s; ++e) M->hnu[e] = F.hnu[e] < 0 ? 0x80 : (uint8_t)F.hnu[e];
    for (int e = 0; e < 4; ++e) M->hnu2 |= (uint32_t)(F.s == 2 ? M->hnu[(e & 1) + 2 * (e >> 1)] : 0) << (8 * e);
    for (int j = 0; j < F.k; ++j) {
        M->taux[j] = (uint8_t)F.ox[j];
        M->tauy[j] = (uint8_t)F.oy[j];
        if (j < 8) {
            M->tx[j / 4] |= (uint32_t)F.ox[j] << (8 * (j % 4));
            M->ty[j / 4] |= (uint32_t)F.oy[j] << (8 * (j % 4));
        }
    }
    M->ds = make_div32((uint32_t)F.s);
    M->dk32 = make_div32((uint32_t)F.k);
    M->dk64 = make_div64((uint64_t)F.k);
    for (int G = 0; G < 4; ++G) {
        // used only when 8G < r: then s^(8G) < n < 2^31 and k^(8G) < N < 2^63
        uint64_t sp = 1, kp = 1;
        for (int i = 0; i < 8 * G && 8 * G < F.r; ++i) {
            sp *= (uint64_t)F.s;
            kp *= (uint64_t)F.k;
        }
        M->dsp[G] = make_div32((uint32_t)sp);
        M->dkp32[G] = make_div32(kp <= 0xFFFFFFFFull ? (uint32_t)kp : 1u);
        M->dkp64[G] = make_div64(kp);
    }
    return M;
}

void mfma_release(FractalHost &F)
{
    delete F.mfma;
    F.mfma = nullptr;
}

static sqz_status mfma_after(const char *what)
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, what);
}

sqz_status launch_lambda_mfma(const FractalHost &F, const uint64_t *idx, int64_t count, int32_t *xy, hipStream_t st)
{
    hipLaunchKernelGGL(k_lambda_mfma, dim3(grid_for_waves((uint64_t)count)), dim3(kBlock), 0, st, *F.mfma, idx, count,
                       xy);
    return mfma_after("lambda_map (mfma) launch");
}

sqz_status launch_nu_mfma(const FractalHost &F, const int32_t *xy, int64_t count, uint64_t *idx, hipStream_t st)
{
    hipLaunchKernelGGL(k_nu_mfma, dim3(grid_for_waves((uint64_t)count)), dim3(kBlock), 0, st, *F.mfma, xy, count, idx);
    return mfma_after("nu_map (mfma) launch");
}

sqz_status launch_life_cell_mfma(const FractalHost &F, const uint8_t *in, uint8_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_life_cell_mfma, dim3(grid_for_waves(F.N)), dim3(kBlock), 0, st, *F.mfma, in, out);
    return mfma_after("compact_step (cell, mfma maps) launch");
}

}  // namespace sqz
