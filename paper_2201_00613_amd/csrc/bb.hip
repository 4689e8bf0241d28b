// Bounding-box baseline (approach "BB" of Section "Experimental Setup and
// Results"): Life on the expanded n x n grid, every hole written 0.
//
// s = 2 fast path: a thread owns a 16-byte wide, kRows-tall column strip and
// slides a three-row window down it, so each input row is fetched once per
// strip (plus two halo rows).  Neighbour counts are byte-wise SIMD-in-register
// sums (counts <= 8 fit a byte); left/right edge bytes come from the
// neighbouring lanes by cross-lane shuffle.  Membership for s = 2: (x, y) is
// a hole iff at some level the bit pair (x_i, y_i) is not a replica offset;
// for a forbidden pair (a, b) that is ((a ? x : ~x) & (b ? y : ~y) & (n-1)) != 0.
#include "common.h"

namespace sqz {

namespace {

constexpr int kBlock = 256;
constexpr int kRows = 16;

struct BBParams {
    uint32_t n;           // side, multiple of 16
    uint32_t strips_x;    // n / 16
    uint32_t forbidden;   // bit (a + 2b) set when (a, b) is not a replica offset
    uint32_t lowmask[16][4];  // member bytes of x = 0..15 for each y mod 16 (low 4 bits only)
};

__device__ __forceinline__ uint32_t align_byte(uint32_t hi, uint32_t lo, uint32_t s)
{
    return __builtin_amdgcn_alignbyte(hi, lo, s);
}

// Byte-wise (t == 3) for bytes t <= 15: 0x01 in each matching byte.
__device__ __forceinline__ uint32_t bytes_eq3(uint32_t t)
{
    uint32_t z = t ^ 0x03030303u;
    uint32_t nz = ((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z;
    return (~nz >> 7) & 0x01010101u;
}

struct Row {
    uint4 d;
    uint32_t l, r;  // byte at x0-1 and at x0+16 (0 outside the box)
};

__device__ __forceinline__ Row load_row(const uint8_t *__restrict__ in, uint32_t n, uint32_t x0, int64_t y, int lane,
                                        bool row_ok)
{
    Row R;
    R.d = make_uint4(0, 0, 0, 0);
    if (row_ok) R.d = *reinterpret_cast<const uint4 *>(in + (uint64_t)y * n + x0);
    // left neighbour byte: top byte of the previous lane's last word
    uint32_t up = __shfl_up(R.d.w, 1);
    uint32_t dn = __shfl_down(R.d.x, 1);
    R.l = up >> 24;
    R.r = dn & 0xFFu;
    const bool first_in_row = x0 == 0, last_in_row = x0 + 16 == n;
    if (lane == 0 || first_in_row) R.l = (!first_in_row && row_ok) ? in[(uint64_t)y * n + x0 - 1] : 0u;
    if (lane == 63 || last_in_row) R.r = (!last_in_row && row_ok) ? in[(uint64_t)y * n + x0 + 16] : 0u;
    return R;
}

// left-shifted (value of x-1) and right-shifted (value of x+1) copies
__device__ __forceinline__ void shifts(const Row &R, uint4 &sl, uint4 &sr)
{
    sl.x = align_byte(R.d.x, R.l << 24, 3);
    sl.y = align_byte(R.d.y, R.d.x, 3);
    sl.z = align_byte(R.d.z, R.d.y, 3);
    sl.w = align_byte(R.d.w, R.d.z, 3);
    sr.x = align_byte(R.d.y, R.d.x, 1);
    sr.y = align_byte(R.d.z, R.d.y, 1);
    sr.z = align_byte(R.d.w, R.d.z, 1);
    sr.w = align_byte(R.r, R.d.w, 1);
}

__global__ void __launch_bounds__(kBlock) k_life_bb2(BBParams B, const uint8_t *__restrict__ in,
                                                     uint8_t *__restrict__ out, uint64_t nthreads)
{
    const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool active = tid < nthreads;
    const uint32_t n = B.n;
    const uint32_t sx = active ? (uint32_t)(tid % B.strips_x) : 0u;
    const uint32_t sy = active ? (uint32_t)(tid / B.strips_x) : 0u;
    const uint32_t x0 = sx * 16;
    const int64_t y0 = (int64_t)sy * kRows;
    const uint32_t nm1 = n - 1;

    Row up = load_row(in, n, x0, y0 - 1, lane, active && y0 > 0);
    Row mid = load_row(in, n, x0, y0, lane, active);
    for (int i = 0; i < kRows; ++i) {
        const int64_t y = y0 + i;
        Row dn = load_row(in, n, x0, y + 1, lane, active && y + 1 < (int64_t)n);
        uint4 ul, ur, ml, mr, dl, dr;
        shifts(up, ul, ur);
        shifts(mid, ml, mr);
        shifts(dn, dl, dr);
        uint4 cnt;
        cnt.x = up.d.x + ul.x + ur.x + ml.x + mr.x + dn.d.x + dl.x + dr.x;
        cnt.y = up.d.y + ul.y + ur.y + ml.y + mr.y + dn.d.y + dl.y + dr.y;
        cnt.z = up.d.z + ul.z + ur.z + ml.z + mr.z + dn.d.z + dl.z + dr.z;
        cnt.w = up.d.w + ul.w + ur.w + ml.w + mr.w + dn.d.w + dl.w + dr.w;
        // membership of the 16 cells of this row segment
        const uint32_t yy = (uint32_t)y;
        bool hole_hi = false;
#pragma unroll
        for (int ab = 0; ab < 4; ++ab)
            if (B.forbidden & (1u << ab)) {
                uint32_t xs = (ab & 1) ? x0 : ~x0;
                uint32_t ys = (ab & 2) ? yy : ~yy;
                hole_hi |= (xs & ys & nm1 & ~15u) != 0;
            }
        const uint32_t *lm = B.lowmask[yy & 15];
        uint4 o;
        o.x = bytes_eq3(cnt.x | mid.d.x) & (hole_hi ? 0u : lm[0]);
        o.y = bytes_eq3(cnt.y | mid.d.y) & (hole_hi ? 0u : lm[1]);
        o.z = bytes_eq3(cnt.z | mid.d.z) & (hole_hi ? 0u : lm[2]);
        o.w = bytes_eq3(cnt.w | mid.d.w) & (hole_hi ? 0u : lm[3]);
        if (active) *reinterpret_cast<uint4 *>(out + (uint64_t)y * n + x0) = o;
        up = mid;
        mid = dn;
    }
}

// Any s: one thread per expanded cell; membership through nu.
__global__ void __launch_bounds__(kBlock) k_life_bb_any(MapParams P, const uint8_t *__restrict__ in,
                                                        uint8_t *__restrict__ out)
{
    const uint64_t n = (uint64_t)P.n, total = n * n;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (uint64_t)gridDim.x * kBlock) {
        const int32_t y = (int32_t)(i / n), x = (int32_t)(i - (uint64_t)y * n);
        uint8_t v = 0;
        if (nu_map(P, x, y) != kHole64) {
            uint32_t cnt = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy) continue;
                    const int32_t qx = x + dx, qy = y + dy;
                    if (qx < 0 || qy < 0 || qx >= (int32_t)n || qy >= (int32_t)n) continue;
                    cnt += in[(uint64_t)qy * n + qx];
                }
            v = (uint8_t)(cnt == 3 || (in[i] && cnt == 2));
        }
        out[i] = v;
    }
}

}  // namespace

sqz_status launch_life_bb(const FractalHost &F, const uint8_t *in, uint8_t *out, hipStream_t st)
{
    const uint64_t n = (uint64_t)F.n;
    if (F.s == 2 && n >= 16) {
        BBParams B;
        B.n = (uint32_t)n;
        B.strips_x = (uint32_t)(n / 16);
        B.forbidden = 0;
        for (int ab = 0; ab < 4; ++ab)
            if (F.hnu[(ab & 1) + 2 * (ab >> 1)] < 0) B.forbidden |= 1u << ab;
        for (uint32_t ylo = 0; ylo < 16; ++ylo)
            for (int w = 0; w < 4; ++w) {
                uint32_t m = 0;
                for (int b = 0; b < 4; ++b) {
                    uint32_t x = 4 * w + b;
                    bool member = true;
                    for (int i = 0; i < 4; ++i) {
                        int xb = (x >> i) & 1, yb = (ylo >> i) & 1;
                        if (F.hnu[xb + 2 * yb] < 0) member = false;
                    }
                    if (member) m |= 1u << (8 * b);
                }
                B.lowmask[ylo][w] = m;
            }
        const uint64_t nthreads = (n / 16) * (n / kRows);
        const uint64_t grid = (nthreads + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_life_bb2, dim3((unsigned)grid), dim3(kBlock), 0, st, B, in, out, nthreads);
    } else {
        uint64_t g = (n * n + kBlock - 1) / kBlock;
        if (g > 16384) g = 16384;
        hipLaunchKernelGGL(k_life_bb_any, dim3((unsigned)g), dim3(kBlock), 0, st, F.P, in, out);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "expanded_step launch");
}

}  // namespace sqz
